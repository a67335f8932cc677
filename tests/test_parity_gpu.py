"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer and byte results (spins, walker maps, flip and exchange counters) and
the binary64 energies and accumulators must be bit-identical: both sides run
the same numeric contract (see the oracle header), and every floating-point
sum on the GPU path is either exact or taken in the oracle's order.  Finalized
observables are bit-identical too: both sides take a disorder average as the
exact sum over samples rounded once, and evaluate each formula in the same
order.
"""
import math

import numpy as np
import pytest

from oracle import ea_oracle as O
from paper_1403_4560_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def gpu_run(work, sweeps, stream=None, plan=None, splits=None, unbatched=False, tier=0):
    from paper_1403_4560_amd import binding
    with binding.Ensemble(work, stream=stream, tier=tier) as ens:
        if plan:
            ens.set_plan(**plan)
        parts = splits or [sweeps]
        assert sum(parts) == sweeps
        for k in parts:
            (ens.sweep_pt_unbatched if unbatched else ens.sweep_pt)(k)
        st = ens.read_state()
        ms = ens.measure()
        bad = ens.check_energies()
    return st, ms, bad


def assert_same(work, st, ms, ref, samples=None):
    samples = range(work.n_samples) if samples is None else samples
    for k, s in enumerate(samples):
        o = ref.states[k]
        assert st["sweep"] == int(o.sweep[0])
        assert np.array_equal(st["walker_at_slot"][s], o.walker_at_slot), ("walker_at_slot", s)
        assert np.array_equal(st["spins"][s], o.spins_slot_order()), ("spins", s)
        assert np.array_equal(st["E"][s], o.energies_slot_order()), ("E", s)
        assert np.array_equal(ms["flips"][s], o.flips), ("flips", s)
        assert np.array_equal(ms["swaps"][s], o.swaps), ("swaps", s)
        assert np.array_equal(ms["acc"][s], o.acc), ("acc", s)


def check(work, sweeps, **kw):
    print("case:", work.name, "S=%d" % work.n_samples, "sweeps=%d" % sweeps, kw, flush=True)
    st, ms, bad = gpu_run(work, sweeps, **kw)
    ref = O.OracleEnsemble(work).run(sweeps)
    assert bad == 0
    assert_same(work, st, ms, ref)
    return st, ms, ref


def test_L4_workload_in_full(torch_cuda):
    # 16 samples, 8 temperatures, 5000 sweeps, measurements every 10 from 2500
    work = W.config_workload("L4_gauss")
    st, ms, ref = check(work, work.sweeps, stream=torch_cuda.cuda.current_stream().cuda_stream)
    assert ms["acc"][0][0, 0] == 250.0


def test_L8_subset_several_tiles(torch_cuda):
    work = W.config_workload("L8_gauss", samples=[0, 5, 1023], measure_start=100)
    check(work, 400, plan=dict(threads=256))


def test_mixed_sizes_and_fields(torch_cuda):
    work = W.config_workload("mixed_L6_12", samples=range(12), measure_start=50)
    check(work, 160)


def test_L16_subset(torch_cuda):
    work = W.config_workload("L16_gauss", samples=[0, 2047], measure_start=0)
    check(work, 40)


def test_pm1_couplings_lds_tier(torch_cuda):
    work = W.make_workload([8, 4, 6], 6, (0.5, 2.0), 0.4, jkind=W.J_PM1, measure_every=5,
                           measure_start=20, name="pm1")
    check(work, 150)
    check(work, 40, tier=2)  # the byte engine at L = 8 too


def test_fields_and_temperatures_at_the_exponent_bounds(torch_cuda):
    # The row and HBM engines split the field into its point on the coupling
    # grid (added to the integer local field, within +-48) and a binary32
    # remainder: a field on the grid (remainder 0), a tiny one, one just inside
    # the grid part's clamp and three beyond it, both signs; temperatures down to
    # 0.002 (beta = 500).  The group engine (L = 6, 10) takes the same fields.
    work = W.make_workload([8, 16, 8, 8, 16, 6, 10, 8], [4, 6, 5, 3, 4, 6, 4, 4], (0.002, 2.0),
                           [0.5, 60.0, -55.0, 47.99, 1e-7, -50.0, 49.0, -0.375], measure_every=4,
                           measure_start=8, name="field bounds")
    check(work, 40)
    check(work.subset([0, 1, 2, 3, 4, 7]), 24, tier=1)  # the HBM tier's half-sweep kernel


def test_bind_buffers_to_caller_memory(torch_cuda):
    # the persistent buffers moved into a torch tensor mid-run: same results
    from paper_1403_4560_amd import binding
    work = W.make_workload([8, 6, 16, 10], [4, 6, 3, 5], (0.5, 2.0), [0.2, 0.1, 0.3, 0.0], measure_every=4,
                           measure_start=4, name="bound")
    need = binding.query_sizes(work)
    print("case: bind_buffers, arena %d bytes" % need, flush=True)
    with binding.Ensemble(work) as ens:
        before = ens.query()["device_bytes"]
        ens.sweep_pt(12)
        with pytest.raises(binding.EAError):
            ens.bind_buffers(torch_cuda.empty(need // 2, dtype=torch_cuda.uint8, device="cuda"))
        arena = torch_cuda.empty(need, dtype=torch_cuda.uint8, device="cuda")
        ens.bind_buffers(arena)
        moved = before - ens.query()["device_bytes"]
        assert 0 < moved <= need < moved + 25 * 256
        with pytest.raises(binding.EAError):
            ens.bind_buffers(arena)
        ens.sweep_pt(20)
        st = ens.read_state()
        ms = ens.measure()
        bad = ens.check_energies()
    ref = O.OracleEnsemble(work).run(32)
    assert bad == 0
    assert_same(work, st, ms, ref)
    del arena


def test_degenerate_sizes(torch_cuda):
    # L = 2 (every neighbour pair joined by two bonds), one temperature (no
    # exchange), an odd number of temperatures, L = 14
    work = W.make_workload([2, 2, 4, 14], [1, 5, 3, 2], (0.5, 2.0), [0.3, 0.0, 0.1, 0.2],
                           measure_every=3, measure_start=5, name="degenerate")
    check(work, 50)


def test_site_engine_forced(torch_cuda):
    # the one-site-per-thread engine (EA_TIER_SITE) for every LDS-resident size
    work = W.make_workload([4, 6, 8, 10, 12, 16], [3, 5, 4, 2, 6, 3], (0.5, 2.0), [0.3, 0.1, 0.2, 0.0, 0.4, 0.1],
                           measure_every=3, measure_start=2, name="site forced")
    check(work, 20, tier=3, plan=dict(chunk=7))
    pm1 = W.make_workload([4, 6, 8], 5, (0.5, 2.0), 0.4, jkind=W.J_PM1, measure_every=2, name="site forced pm1")
    check(pm1, 20, tier=3)


def test_group_engine_quads_and_fields(torch_cuda):
    # walker-interleaved engine: partial quads (n_T = 1, 2, 3, 5, 7), full ones
    # (4, 16), the Table I ladder length (56), both coupling kinds; L = 4 with
    # 32 temperatures has enough work items for it, L = 2 and 4 with few do not
    work = W.make_workload([6, 10, 12, 14, 4, 2, 6, 4], [1, 2, 3, 5, 7, 16, 56, 32], (0.5, 2.0),
                           [0.1, 0.3, -0.2, 0.0, 0.4, 0.2, 0.1, 0.3], measure_every=4, measure_start=1,
                           name="group quads")
    check(work, 12, plan=dict(chunk=5))
    pm1 = W.make_workload([6, 10, 4, 12], [56, 3, 5, 16], (0.5, 2.0), [0.1, 0.4, -0.3, 2.0], jkind=W.J_PM1,
                          measure_every=3, name="group quads pm1")
    check(pm1, 10, splits=[4, 6])


def test_group_engine_tally_forms(torch_cuda):
    """The group engine sums its per-walker tallies in one of three forms: four
    quads with at most five site groups per thread and half-sweep (bytes and
    int32 over a residue class of four lanes), other teams of four or more
    waves with one, two or four quads (16-bit lanes and int64 over a row of
    16), and per thread otherwise.  L = 14 with 16 and 13 temperatures (three
    site groups per thread, padding walkers in the last quad) takes the first,
    L = 12 with 6 temperatures (two quads) the second on teams of 256 or more
    threads, L = 12 with 10 (three quads) the third, L = 10 with 16 the first
    or the third by team size; under every team plan the batch launch allows
    (and per class launch) each equals the oracle bit for bit."""
    from paper_1403_4560_amd import binding
    work = W.make_workload([14, 14, 12, 12, 10], [16, 13, 6, 10, 16], (0.5, 1.6), [0.1, 0.2, 0.3, -0.1, 0.2],
                           measure_every=3, measure_start=1, name="tally forms")
    sweeps = 9
    ref = O.OracleEnsemble(work).run(sweeps)
    with binding.Ensemble(work) as ens:
        assert ens.get_plan().batch == 1
        variants = batch_variants(ens)
    for teams in variants + [None]:
        print("case: tally forms, batch plan", teams, flush=True)
        with binding.Ensemble(work) as ens:
            if teams is None:
                ens.set_plan(batch=False)
            else:
                ens.set_batch_plan(teams)
            ens.set_plan(chunk=4)
            ens.sweep_pt(sweeps)
            st = ens.read_state()
            ms = ens.measure()
            assert ens.check_energies() == 0
        assert_same(work, st, ms, ref)


def test_group_engine_unbatched(torch_cuda):
    work = W.config_workload("mixed_L6_12", samples=[0, 2, 3], measure_start=4)
    check(work, 16, unbatched=True)


def test_never_measure(torch_cuda):
    work = W.make_workload([4, 6], 4, (0.5, 2.0), 0.3, measure_every=0, name="m0")
    st, ms, ref = check(work, 30)
    assert all((a == 0).all() for a in ms["acc"])


@pytest.mark.parametrize("plan", [dict(threads=256, chunk=1, use_graph=0),
                                  dict(threads=512, chunk=7, use_graph=1),
                                  dict(threads=1024, chunk=100, use_graph=0),
                                  dict(threads=1024, chunk=13, use_graph=1)])
def test_plan_invariance(torch_cuda, plan):
    work = W.config_workload("mixed_L6_12", samples=[0, 1, 2, 3, 16, 17], measure_start=10)
    check(work, 45, plan=plan)


def test_chunking_invariance(torch_cuda):
    work = W.config_workload("L8_gauss", samples=[3, 4], measure_start=30)
    check(work, 100, splits=[37, 1, 62], plan=dict(chunk=16))


def test_unbatched_equals_oracle(torch_cuda):
    work = W.config_workload("L8_gauss", samples=[7, 8, 9], measure_start=20)
    check(work, 60, unbatched=True)


def test_batch_invariance(torch_cuda):
    work = W.config_workload("mixed_L6_12", samples=range(8), measure_start=0)
    st_all, ms_all, _ = gpu_run(work, 30)
    one = work.subset([5])
    st_one, ms_one, _ = gpu_run(one, 30)
    assert np.array_equal(st_all["spins"][5], st_one["spins"][0])
    assert np.array_equal(ms_all["acc"][5], ms_one["acc"][0])


def _resume_cases():
    return [W.config_workload("L8_gauss", samples=[11, 12], measure_start=10),
            W.make_workload([12, 6], [16, 5], (0.5, 1.6), [0.1, 0.3], measure_start=10, name="group resume"),
            W.make_workload([32, 8, 10], [4, 6, 7], (0.5, 2.0), 0.4, jkind=W.J_PM1, measure_start=10,
                            name="bits+group pm1 resume")]


@pytest.mark.parametrize("with_map", [True, False])
@pytest.mark.parametrize("case", range(3))
def test_checkpoint_resume(torch_cuda, case, with_map):
    # with the walker map the resumed run continues the interrupted one exactly,
    # walker labels included; without it walkers are renumbered by slot, which
    # changes nothing else (random numbers are keyed by slot)
    from paper_1403_4560_amd import binding
    work = _resume_cases()[case]
    print("case:", work.name, "walker map" if with_map else "no walker map", flush=True)
    st_full, ms_full, _ = gpu_run(work, 80)
    with binding.Ensemble(work) as a:
        a.sweep_pt(35)
        st = a.read_state()
        ms = a.measure()
    assert any((np.asarray(w) != np.arange(w.shape[1])).any() for w in st["walker_at_slot"])
    with binding.Ensemble(work) as b:
        b.write_state(st["spins"], st["sweep"], walker_at_slot=st["walker_at_slot"] if with_map else None)
        b.load_accumulators(ms["acc"], ms["flips"], ms["swaps"])
        b.sweep_pt(45)
        st2 = b.read_state()
        ms2 = b.measure()
        assert b.check_energies() == 0
    for s in range(work.n_samples):
        assert np.array_equal(st2["spins"][s], st_full["spins"][s])
        assert np.array_equal(st2["E"][s], st_full["E"][s])
        assert np.array_equal(ms2["acc"][s], ms_full["acc"][s])
        assert np.array_equal(ms2["flips"][s], ms_full["flips"][s])
        assert np.array_equal(ms2["swaps"][s], ms_full["swaps"][s])
        if with_map:
            assert np.array_equal(st2["walker_at_slot"][s], st_full["walker_at_slot"][s])


def test_write_state_rejects_a_walker_map_that_is_not_a_permutation(torch_cuda):
    from paper_1403_4560_amd import binding
    work = W.make_workload([4, 6], [3, 5], (0.5, 2.0), 0.2, name="bad map")
    with binding.Ensemble(work) as ens:
        st = ens.read_state()
        bad = [w.copy() for w in st["walker_at_slot"]]
        bad[1][0, 1] = bad[1][0, 0]
        with pytest.raises(binding.EAError):
            ens.write_state(st["spins"], st["sweep"], walker_at_slot=bad)
        bad[1][0, 1] = 5
        with pytest.raises(binding.EAError):
            ens.write_state(st["spins"], st["sweep"], walker_at_slot=bad)
        ens.write_state(st["spins"], st["sweep"], walker_at_slot=st["walker_at_slot"])
        assert ens.check_energies() == 0


def test_measure_now_matches_oracle(torch_cuda):
    from paper_1403_4560_amd import binding
    work = W.make_workload([6, 4], 3, (0.5, 2.0), 0.2, measure_every=0, name="now")
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(12)
        st = ens.read_state()
        ms = ens.measure(now=True)
    for s in range(2):
        L = int(work.L[s])
        for t in range(int(work.n_temps[s])):
            acc, _ = O.measure_pair(L, st["spins"][s][0, t], st["spins"][s][1, t],
                                    st["E"][s][0, t], st["E"][s][1, t])
            assert np.array_equal(ms["acc"][s][t], acc)


def same_obs(gpu, ref, names=None):
    """Bitwise equality of finalized observables (NaN where both are NaN)."""
    for k in (names or [n for n in O.OBS_NAMES]):
        a, b = np.asarray(gpu[k]), np.asarray(ref[k])
        assert np.array_equal(a, b, equal_nan=True), (k, a, b)


def test_finalize_matches_oracle(torch_cuda):
    from paper_1403_4560_amd import binding
    work = W.config_workload("L4_gauss", measure_start=200)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(1200)
        ms = ens.measure()
        fin = ens.finalize()
        jk = ens.finalize_jackknife()
    acc = np.stack(ms["acc"])
    ref = O.observables(acc, 4)
    assert np.all(fin["n_samples"] == 16)
    same_obs(fin, ref)
    rjk = O.jackknife(acc, 4)
    same_obs({k: v[0] for k, v in jk.items()}, {k: v[0] for k, v in rjk.items()})
    same_obs({k: v[1] for k, v in jk.items()}, {k: v[1] for k, v in rjk.items()})


def test_finalize_one_system_per_selection(torch_cuda):
    """A mixed batch (four lattice sizes, three fields): each (L, h) system
    finalized on its own, bit-identical to the oracle; a selection that mixes
    fields, sizes or ladders is refused."""
    from paper_1403_4560_amd import binding
    work = W.config_workload("mixed_L6_12", samples=range(36), measure_start=20)
    sweeps = 60
    print("case: finalize per system, mixed 36 samples, %d sweeps" % sweeps, flush=True)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(sweeps)
        ms = ens.measure()
        systems = ens.systems()
        got = [(sel, ens.finalize(sel), ens.finalize_jackknife(sel)) for sel in systems]
        h = np.asarray(work.h)
        L = np.asarray(work.L)
        six = [s for s in range(work.n_samples) if L[s] == 6]
        mixed_field = [six[0], next(s for s in six if h[s] != h[six[0]])]
        for bad in (mixed_field, [0, 1], None, [0, 0], [work.n_samples]):
            with pytest.raises(binding.EAError):
                ens.finalize(bad)
        with pytest.raises(binding.EAError):
            ens.finalize_jackknife(systems[0][:1])
    assert len(systems) == 12 and sorted(sum(systems, [])) == list(range(work.n_samples))
    ref = O.OracleEnsemble(work).run(sweeps)
    acc = np.stack([st.acc for st in ref.states])
    for s in range(work.n_samples):
        assert np.array_equal(ms["acc"][s], acc[s]), s
    for sel, fin, jk in got:
        Ls = {int(L[s]) for s in sel}
        hs = {float(h[s]) for s in sel}
        assert len(Ls) == 1 and len(hs) == 1
        Lsys = Ls.pop()
        same_obs(fin, O.observables(acc[sel], Lsys))
        rjk = O.jackknife(acc[sel], Lsys)
        same_obs({k: v[0] for k, v in jk.items()}, {k: v[0] for k, v in rjk.items()})
        same_obs({k: v[1] for k, v in jk.items()}, {k: v[1] for k, v in rjk.items()})
        assert np.all(fin["n_samples"] == len(sel))


def adversarial_accumulators(S, nT, seed):
    """Accumulators whose disorder sums defeat ordinary summation: thermal
    means spread over many binades, near-cancelling pairs, subnormals, values
    near the overflow threshold, zero measurement counts and infinities."""
    rng = np.random.default_rng(seed)
    acc = np.zeros((S, nT, O.NACC))
    acc[..., 0] = rng.integers(1, 2000, size=(S, nT)).astype(np.float64)
    mag = 10.0 ** rng.integers(-30, 30, size=(S, nT, O.NACC - 1))
    acc[..., 1:] = rng.normal(size=(S, nT, O.NACC - 1)) * mag * acc[..., :1]
    acc[1, :, 1:] = -acc[0, :, 1:] * (acc[1, :, :1] / acc[0, :, :1])      # sample 1 cancels sample 0
    acc[2, 0, 5:9] = [5e-324, -1e-320, 2.2250738585072014e-308, 4e-310]      # subnormal means (n = ..)
    acc[2, 0, 0] = 1.0
    acc[3, 1, 7:10] = [1.7e308, 1.7e308, -1.7e308]                           # near overflow
    acc[3, 1, 0] = 1.0
    if nT > 2:
        acc[4, 2, :] = 0.0                                                   # never measured: NaN means
        acc[5, 2, 12] = np.inf
    return acc


@pytest.mark.parametrize("S,seed", [(7, 1), (40, 2)])
def test_finalize_exact_sums_on_adversarial_accumulators(torch_cuda, S, seed):
    """Loaded accumulators chosen against ordinary summation: the device's
    exact sums, rounded once, equal the oracle's bit for bit (observables and
    jackknife errors), and do not depend on the order of the selection."""
    from paper_1403_4560_amd import binding
    nT, L = 4, 6
    work = W.make_workload([L] * S, nT, (0.5, 2.0), 0.2, name="adversarial")
    acc = adversarial_accumulators(S, nT, seed)
    print("case: adversarial finalize S=%d seed=%d" % (S, seed), flush=True)
    with binding.Ensemble(work) as ens:
        ens.load_accumulators(acc=[acc[s] for s in range(S)])
        fin = ens.finalize()
        jk = ens.finalize_jackknife()
        perm = np.random.default_rng(seed).permutation(S)
        jk_perm = ens.finalize_jackknife(perm)
    same_obs(fin, O.observables(acc, L))
    rjk = O.jackknife(acc, L)
    for got in (jk, jk_perm):
        same_obs({k: v[0] for k, v in got.items()}, {k: v[0] for k, v in rjk.items()})
        same_obs({k: v[1] for k, v in got.items()}, {k: v[1] for k, v in rjk.items()})


def test_failed_frame_allocation_leaves_the_ensemble_usable(torch_cuda):
    """A chunk whose snapshot frames cannot be allocated fails with
    EA_ENOMEM and leaves the ensemble as it was (old frames and capacity):
    a following run with a small chunk gives the oracle's results."""
    from paper_1403_4560_amd import binding
    work = W.config_workload("L16_gauss", samples=range(160), measure_every=1, measure_start=0)
    frame_bytes = sum(2 * int(nT) * int(L) * int(L) * 4 for L, nT in zip(work.L, work.n_temps))
    need = (100000 + 2) * frame_bytes
    total = torch_cuda.cuda.get_device_properties(0).total_memory
    assert need > 1.5 * total, "the workload must ask for more frame memory than the device has"
    print("case: frame allocation of %.0f GB refused, then chunk 7" % (need / 1e9), flush=True)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(3)
        ens.set_plan(chunk=100000)
        with pytest.raises(binding.EAError) as err:
            ens.sweep_pt(100000)
        assert err.value.status == -2
        ens.set_plan(chunk=7)
        ens.sweep_pt(9)
        st = ens.read_state()
        ms = ens.measure()
        bad = ens.check_energies()
    assert bad == 0
    ref = O.OracleEnsemble(work.subset([0, 159])).run(12)
    assert_same(work, st, ms, ref, samples=[0, 159])


def test_full_L16_workload_sampled(torch_cuda):
    """The 2048-sample, 24-temperature L = 16 batch in the benchmark's launch
    configuration; samples compared one by one against the oracle."""
    from paper_1403_4560_amd import binding
    work = W.config_workload("L16_gauss", measure_start=0)
    sweeps = 20
    print("case: full L16 batch, 2048 samples, %d sweeps" % sweeps, flush=True)
    with binding.Ensemble(work) as ens:
        ens.set_plan(chunk=10)
        ens.sweep_pt(sweeps)
        st = ens.read_state()
        ms = ens.measure()
        assert ens.check_energies() == 0
    pick = [0, 777, 2047]
    ref = O.OracleEnsemble(work.subset(pick)).run(sweeps)
    assert_same(work, st, ms, ref, samples=pick)


def test_full_L8_workload_sampled(torch_cuda):
    """The whole 1024-sample, 16-temperature L = 8 batch in the benchmark's
    plan (graph replay), measuring from the first sweep; three samples spread
    over the batch compared one by one against the oracle."""
    from paper_1403_4560_amd import binding
    work = W.config_workload("L8_gauss", measure_start=0)
    sweeps = 20
    print("case: full L8 batch, 1024 samples, %d sweeps" % sweeps, flush=True)
    with binding.Ensemble(work) as ens:
        ens.set_plan(chunk=10)
        ens.sweep_pt(sweeps)
        st = ens.read_state()
        ms = ens.measure()
        assert ens.check_energies() == 0
    pick = [0, 511, 1023]
    ref = O.OracleEnsemble(work.subset(pick)).run(sweeps)
    assert_same(work, st, ms, ref, samples=pick)


def test_full_mixed_workload_sampled(torch_cuda):
    """The whole 4096-sample mixed batch (L = 6, 8, 10, 12; h = 0.1, 0.2,
    0.3), measuring from the first sweep; two samples of every lattice size at
    two different fields, from both ends of the batch, against the oracle."""
    from paper_1403_4560_amd import binding
    work = W.config_workload("mixed_L6_12", measure_start=0)
    sweeps = 20
    print("case: full mixed batch, 4096 samples, %d sweeps" % sweeps, flush=True)
    with binding.Ensemble(work) as ens:
        ens.set_plan(chunk=10)
        ens.sweep_pt(sweeps)
        st = ens.read_state()
        ms = ens.measure()
        assert ens.check_energies() == 0
    pick = [0, 4, 9, 13, 4094, 4087, 4092, 4091, 2050]
    assert len({(int(work.L[s]), float(work.h[s])) for s in pick}) == 8
    ref = O.OracleEnsemble(work.subset(pick)).run(sweeps)
    assert_same(work, st, ms, ref, samples=pick)


@pytest.mark.parametrize("name,pick", [("L16_gauss", [1, 1024, 2046]),
                                       ("mixed_L6_12", [2, 7, 4093, 4088, 1029, 2051])])
def test_full_workload_in_the_bench_plan(torch_cuda, name, pick):
    """The whole batch exactly as bench.py times it: autotuned plan, chunks of
    100 sweeps replayed from a hipGraph, measurements from the first sweep;
    200 sweeps, samples spread over the batch compared with the oracle."""
    from paper_1403_4560_amd import binding
    work = W.config_workload(name, measure_start=0)
    sweeps = 200
    print("case: %s whole batch in the bench plan, %d sweeps" % (name, sweeps), flush=True)
    with binding.Ensemble(work) as ens:
        ens.autotune(trial_sweeps=2)
        ens.set_plan(chunk=100, use_graph=True)
        ens.sweep_pt(sweeps)
        st = ens.read_state()
        ms = ens.measure()
        assert ens.check_energies() == 0
    ref = O.OracleEnsemble(work.subset(pick)).run(sweeps)
    assert_same(work, st, ms, ref, samples=pick)


def test_L16_long_run_in_the_bench_plan(torch_cuda):
    """Two L = 16 samples for 600 sweeps in the benchmark's plan (chunks of 100
    replayed from a hipGraph), measuring every 10 sweeps from 300: spins,
    walker maps, energies, counters and accumulators equal the oracle's."""
    work = W.config_workload("L16_gauss", samples=[5, 1500], measure_start=300)
    check(work, 600)


def test_L32_pm1_longer_run(torch_cuda):
    work = W.config_workload("L32_pm1", samples=[3], measure_start=20)
    check(work, 60)


def test_invalid_plan_rejected(torch_cuda):
    from paper_1403_4560_amd import binding
    work = W.make_workload([4], 2, (0.5, 2.0), 0.3)
    with binding.Ensemble(work) as ens:
        with pytest.raises(binding.EAError):
            ens.set_plan(threads=300)
        with pytest.raises(binding.EAError):
            ens.set_plan(chunk=0)
        with pytest.raises(binding.EAError):
            ens.sweep_pt(-1)


def test_fast_exponential_bracket_is_exhaustively_safe(torch_cuda):
    from paper_1403_4560_amd import binding
    v, dev = binding.verify_exp_bracket()
    print("bracket: violations=%d max relative deviation=%.3g" % (v, dev), flush=True)
    assert v == 0
    assert dev < 2.0 ** -13


def test_exchange_shortcut_is_exhaustively_safe(torch_cuda):
    # the exchange test decides u53 < exp_ea64(D) from the hardware exponential
    # outside a relative margin of 2^-16; with the rounding of its argument
    # (1.32e-6) the bounds checked here keep it inside 1.7e-6
    from paper_1403_4560_amd import binding
    v, dev = binding.verify_exchange_bracket()
    print("exchange bracket: violations=%d max relative deviation=%.3g" % (v, dev), flush=True)
    assert v == 0
    assert dev <= 2.0 ** -22
    assert 2.0 ** -19 * math.log(2.0) * 1.001 + dev + 2.0 ** -49 < 1.7e-6 < 2.0 ** -16


def test_autotune_keeps_results(torch_cuda, monkeypatch):
    from paper_1403_4560_amd import binding
    monkeypatch.delenv("EA_TUNE_CACHE", raising=False)
    work = W.config_workload("mixed_L6_12", samples=[0, 1, 2, 3], measure_start=0)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(7)
        plan = ens.autotune(trial_sweeps=3)
        assert plan.threads in (256, 512, 1024) and plan.batch in (0, 1)
        ens.sweep_pt(13)
        st = ens.read_state()
        ms = ens.measure()
    ref = O.OracleEnsemble(work).run(20)
    assert_same(work, st, ms, ref)


# --- the batch launch: every lattice-size class of the small engines in one
# persistent launch, units of up to P items per workgroup --------------------
def batch_variants(ens):
    """Team plans to try: the default, and the largest and the smallest
    possible teams per workgroup for every batch class."""
    from paper_1403_4560_amd import binding
    base = list(ens.batch_plan()["teams"])
    cands = []
    for i, p in enumerate(base):
        if p == 0:
            cands.append([0])
            continue
        ok = []
        for P in (1, 2, 4, 8):
            t = list(base)
            t[i] = P
            try:
                ens.set_batch_plan(t)
                ok.append(P)
            except binding.EAError:
                pass
        cands.append(ok)
    ens.set_batch_plan(base)
    return [base, [max(c) for c in cands], [min(c) for c in cands]]


@pytest.mark.parametrize("jkind", [W.J_GAUSS, W.J_PM1])
def test_batch_launch_plans_match_oracle(torch_cuda, jkind):
    """Uneven sizes and ladder lengths (group engine at L = 6, 10, 12, row
    engine at L = 8 for Gaussian couplings, site engine at L = 4), as one batch
    launch with several team plans (ghost teams included) and as one launch
    per class: every plan equals the oracle bit for bit."""
    from paper_1403_4560_amd import binding
    Ls = [6, 8, 10, 12, 4, 6, 8, 12, 10, 6, 4, 6, 6]
    nT = [16, 16, 16, 16, 8, 5, 13, 16, 7, 16, 3, 16, 16]
    hs = [0.1, 0.2, 0.3, 0.1, 0.2, 0.3, 0.1, 0.2, 0.3, 0.1, 0.2, 0.3, 0.0]
    work = W.make_workload(Ls, nT, (0.5, 1.6), hs, jkind=jkind, measure_every=4, measure_start=4,
                           name="batch plans")
    sweeps = 18
    ref = O.OracleEnsemble(work).run(sweeps)
    with binding.Ensemble(work) as ens:
        assert ens.get_plan().batch == 1
        variants = batch_variants(ens)
    assert any(v != variants[0] for v in variants[1:])
    for teams in variants + [None]:
        print("case: batch plan", teams, "jkind", jkind, flush=True)
        with binding.Ensemble(work) as ens:
            if teams is None:
                ens.set_plan(batch=False)
            else:
                ens.set_batch_plan(teams)
            ens.set_plan(chunk=7)
            ens.sweep_pt(sweeps)
            st = ens.read_state()
            ms = ens.measure()
            assert ens.check_energies() == 0
        assert_same(work, st, ms, ref)


def test_autotune_plan_cache(torch_cuda, tmp_path, monkeypatch):
    """The autotuner stores its plan under the ensemble's signature and a
    second ensemble of the same shape takes it from the cache; results are
    unchanged."""
    from paper_1403_4560_amd import binding
    cache = tmp_path / "plans.txt"
    monkeypatch.setenv("EA_TUNE_CACHE", str(cache))
    work = W.config_workload("mixed_L6_12", samples=range(16), measure_start=0)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(5)
        p1 = ens.autotune(trial_sweeps=2)
        b1 = ens.batch_plan()
        ens.sweep_pt(9)
        st = ens.read_state()
        ms = ens.measure()
    text = cache.read_text()
    assert text.startswith(b1["signature"] + " batch=%d threads=%d P=" % (p1.batch, p1.threads))
    ref = O.OracleEnsemble(work).run(14)
    assert_same(work, st, ms, ref)
    with binding.Ensemble(work) as ens2:
        other = [0 if t == 0 else 1 for t in b1["teams"]]
        ens2.set_batch_plan(other)
        p2 = ens2.autotune(trial_sweeps=2)      # from the cache: no timing
        assert ens2.batch_plan()["teams"] == b1["teams"] and p2.batch == p1.batch
    assert cache.read_text() == text


# --- multispin (one bit per spin) engine, +-1 couplings at L = 8, 16, 32 -------
def test_bits_engine_sizes_and_fields(torch_cuda):
    # n_T = 1 (no exchange), odd n_T and lane groups that leave idle lanes;
    # h = 0 (k_+ = k_- = 3), h = 0.4 and -0.3, |h| > 6 (one spin sign never
    # lowers the energy, the other always does) and a tiny field
    Ls = [8, 8, 16, 16, 32, 8, 16, 32, 8]
    nT = [1, 5, 3, 24, 2, 17, 7, 3, 4]
    hs = [0.0, 0.4, -0.3, 0.4, 0.4, 7.0, -6.5, 1e-3, 2.0]
    work = W.make_workload(Ls, nT, (0.5, 2.0), hs, jkind=W.J_PM1, measure_every=3, measure_start=2,
                           name="bits sizes/fields")
    check(work, 25, plan=dict(chunk=9))


def test_bits_engine_equals_byte_engines(torch_cuda):
    work = W.make_workload([8, 16, 32], [6, 5, 4], (0.5, 2.0), [0.4, 0.1, -0.2], jkind=W.J_PM1,
                           measure_every=2, measure_start=0, name="bits vs bytes")
    st_b, ms_b, bad_b = gpu_run(work, 14)
    st_y, ms_y, bad_y = gpu_run(work, 14, tier=2)
    assert bad_b == 0 and bad_y == 0
    for s in range(work.n_samples):
        assert np.array_equal(st_b["spins"][s], st_y["spins"][s])
        assert np.array_equal(st_b["E"][s], st_y["E"][s])
        assert np.array_equal(ms_b["acc"][s], ms_y["acc"][s])
        assert np.array_equal(ms_b["flips"][s], ms_y["flips"][s])


def test_bits_engine_unbatched_and_resume(torch_cuda):
    work = W.make_workload([32, 16], [4, 6], (0.5, 2.0), 0.4, jkind=W.J_PM1, sample_ids=[9, 3],
                           measure_every=4, measure_start=1, name="bits unbatched")
    check(work, 11, unbatched=True)
    check(work, 11, splits=[4, 7], plan=dict(chunk=3))


# --- HBM-resident tier --------------------------------------------------------
def test_hbm_L32_pm1_subset(torch_cuda):
    work = W.config_workload("L32_pm1", samples=[0, 511], measure_start=0, measure_every=5)
    check(work, 16, tier=1)


def test_hbm_forced_gaussian_L8_L16(torch_cuda):
    work = W.make_workload([8, 16, 8], [16, 6, 3], (0.5, 2.0), [0.2, 0.1, 0.3], measure_every=4,
                           measure_start=3, name="forced-hbm")
    check(work, 30, tier=1)


def test_hbm_L24_gaussian_and_mixed_tiers(torch_cuda):
    work = W.make_workload([24, 4, 8], [4, 5, 6], (0.5, 2.0), [0.2, 0.1, 0.3], measure_every=3,
                           measure_start=2, name="L24+lds")
    check(work, 14, plan=dict(chunk=5))


def test_hbm_mixed_tiers_pm1(torch_cuda):
    work = W.make_workload([32, 4, 8, 16], [3, 4, 5, 6], (0.5, 2.0), 0.4, jkind=W.J_PM1, measure_every=2,
                           measure_start=0, name="pm1 L32+lds")
    check(work, 12, splits=[5, 7], plan=dict(chunk=4))


def test_hbm_unbatched_equals_oracle(torch_cuda):
    work = W.make_workload([32, 32], 4, (0.5, 2.0), 0.4, jkind=W.J_PM1, sample_ids=[5, 6], measure_every=3,
                           measure_start=0, name="pm1 unbatched")
    check(work, 9, unbatched=True, tier=1)


def test_full_L32_workload_sampled(torch_cuda):
    """The 512-sample, 32-temperature L = 32 batch with +-1 couplings."""
    from paper_1403_4560_amd import binding
    work = W.config_workload("L32_pm1", measure_start=0)
    sweeps = 10
    print("case: full L32 batch, 512 samples, %d sweeps" % sweeps, flush=True)
    with binding.Ensemble(work) as ens:
        ens.set_plan(chunk=10)
        ens.sweep_pt(sweeps)
        st = ens.read_state()
        ms = ens.measure()
        assert ens.check_energies() == 0
    pick = [0, 300]
    ref = O.OracleEnsemble(work.subset(pick)).run(sweeps)
    assert_same(work, st, ms, ref, samples=pick)


def test_row_engine_partial_waves(torch_cuda):
    # n_T not a multiple of the walkers a wave holds (4 at L = 16, 16 at L = 8):
    # idle lanes share waves with working ones
    work = W.make_workload([16, 16, 16, 8, 8], [1, 5, 23, 3, 17], (0.4, 1.5), [0.1, 0.2, 0.0, 0.3, 0.1],
                           measure_every=4, measure_start=2, name="row partial waves")
    check(work, 18, plan=dict(chunk=6))


def test_engine_routing(torch_cuda):
    """Which engine each sample runs on, by size, coupling kind, field and tier."""
    from paper_1403_4560_amd import binding
    gauss = W.make_workload([16, 8, 12, 6, 4, 2, 24, 16], [24, 16, 16, 16, 8, 3, 2, 64], (0.5, 2.0), 0.1,
                            name="routing gauss")
    with binding.Ensemble(gauss) as e:
        # L = 4 with 8 temperatures has too few (quad, site group) items for the
        # group engine; L = 16 with 64 temperatures does not fit LDS at all
        assert e.engines() == ["row", "row", "group", "group", "site", "site", "hbm", "hbm"]
    with binding.Ensemble(gauss.subset([0, 1, 2]), tier=3) as e:
        assert e.engines() == ["site"] * 3
    with binding.Ensemble(gauss.subset([0, 1]), tier=1) as e:
        assert e.engines() == ["hbm"] * 2
    pm1 = W.make_workload([32, 16, 8, 10, 32], [32, 24, 16, 56, 40], (0.5, 2.0), 0.4, jkind=W.J_PM1,
                          name="routing pm1")
    with binding.Ensemble(pm1) as e:
        # 40 temperatures at L = 32 do not fit LDS at one bit per spin
        assert e.engines() == ["bits", "bits", "bits", "group", "hbm"]
    with binding.Ensemble(pm1.subset([0, 1, 2]), tier=2) as e:
        assert e.engines() == ["hbm", "group", "group"]


def test_measure_peaks_runs(torch_cuda):
    # the roofline's unit rates: positive, and below twice what 256 CUs of four
    # 16-lane SIMDs at 2.4 GHz give (simple operations measure above the 1x figure)
    from paper_1403_4560_amd import binding
    r = binding.measure_peaks()
    print("peaks:", {k: "%.3g" % v for k, v in r.items()}, flush=True)
    for k in ("valu_xor_ops", "valu_mad_u64_ops", "valu_mul_hi_ops", "valu_exp_ops"):
        assert 0 < r[k] < 2 * 256 * 64 * 2.4e9
    assert 0 < r["lds_read_bytes"] and 0 < r["hbm_copy_bytes"] < 2e13
