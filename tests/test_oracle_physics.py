"""Pins of the oracle's dynamics and measurements against mathematics.

Each check is independent of the oracle's own code:
* exact enumeration of the L = 2 lattice (2^8 states, each of the 24 periodic
  bonds independent) gives the Boltzmann averages of E, q(0) moments and
  |q(k)|^2 at each temperature, and the exact replica-exchange acceptance
  rate; the Monte Carlo averages of independent runs must agree within 5
  standard errors (Methods: eq. 1, parallel tempering, eqs. 2-4);
* with all couplings zero every spin is independent: m = tanh(beta h),
  <q> = m^2, chi = 1 - m^4;
* the energy the sweep tracks incrementally equals a from-scratch evaluation
  of eq. 1 written here with numpy rolls, exactly (couplings on a 2^-18 grid);
* q(k) from the oracle's plane sums equals the discrete Fourier transform of
  the overlap field computed by numpy.fft.
"""
import math

import numpy as np
import pytest

from oracle import ea_oracle as O
from paper_1403_4560_amd import workload as W


def hamiltonian(L, J, s, h):
    """eq. 1 by lattice rolls: bond d of site (z,y,x) joins it to site + d."""
    s3 = s.reshape(L, L, L).astype(np.float64)
    J3 = np.asarray(J, dtype=np.float64).reshape(3, L, L, L)
    EJ = -(J3[0] * s3 * np.roll(s3, -1, axis=2)).sum() \
         - (J3[1] * s3 * np.roll(s3, -1, axis=1)).sum() \
         - (J3[2] * s3 * np.roll(s3, -1, axis=0)).sum()
    M = s3.sum()
    return EJ, M, EJ - h * M


def all_states(N):
    idx = np.arange(2 ** N)
    return np.where((idx[:, None] >> np.arange(N)[None, :]) & 1, -1, 1).astype(np.int8)


def enumerate_L2(J, h, betas):
    L, N = 2, 8
    S = all_states(N)
    E = np.array([hamiltonian(L, J, s, h)[2] for s in S])
    x = np.arange(N) % L
    y = (np.arange(N) // L) % L
    phase_x = np.where(x == 1, -1.0, 1.0)          # e^{i pi x}
    phase_d = np.where((x + y) % 2 == 1, -1.0, 1.0)  # e^{i pi (x+y)}
    Sf = S.astype(np.float64)
    Q0 = Sf @ Sf.T / N
    Qx = (Sf * phase_x) @ Sf.T / N
    Qd = (Sf * phase_d) @ Sf.T / N
    out = []
    for b in betas:
        w = np.exp(-b * (E - E.min()))
        pi = w / w.sum()
        avg = lambda F: pi @ F @ pi
        out.append(dict(pi=pi, E=pi @ E, q1=avg(Q0), q2=avg(Q0 ** 2), q4=avg(Q0 ** 4),
                        kx2=avg(Qx ** 2), kd2=avg(Qd ** 2)))
    return E, out


def run_independent(L, n_T, betas, h, jkind, J, runs, sweeps, burn, mode, seed=11):
    states = []
    for r in range(runs):
        spins0 = W.initial_spins(seed, 1000 + r, L, n_T)
        st = O.SampleState(L, n_T, betas, h, jkind, J, spins0, seed, r,
                           measure_every=1, measure_start=burn, mode=mode)
        states.append(st)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        list(ex.map(lambda st: st.run(sweeps), states))
    return states


def check(mc, exact, what):
    mc = np.asarray(mc)
    mean = mc.mean()
    se = mc.std(ddof=1) / math.sqrt(len(mc))
    assert abs(mean - exact) <= 5.0 * se + 1e-9, (what, mean, exact, se)


@pytest.mark.parametrize("jkind,mode", [(W.J_GAUSS, O.MODE_MIRROR), (W.J_PM1, O.MODE_MIRROR),
                                        (W.J_GAUSS, O.MODE_FP64)])
def test_equilibrium_L2_enumeration(jkind, mode):
    L, n_T, h = 2, 4, 0.3
    betas = W.geometric_betas(n_T, 0.5, 2.0)
    J = (W.gaussian_couplings(5, 0, L) if jkind == W.J_GAUSS else W.pm1_couplings(5, 0, L))
    h32 = float(np.float32(h))
    _, ex = enumerate_L2(J, h32, betas)
    sts = run_independent(L, n_T, betas, h, jkind, J, runs=16, sweeps=20000, burn=1000, mode=mode)
    for t in range(n_T):
        m = [st.acc[t] / st.acc[t, 0] for st in sts]
        check([a[32] for a in m], ex[t]["E"], ("E_a", t))
        check([a[34] for a in m], ex[t]["E"], ("E_b", t))
        check([a[1] for a in m], ex[t]["q1"], ("q", t))
        check([a[2] for a in m], ex[t]["q2"], ("q2", t))
        check([a[4] for a in m], ex[t]["q4"], ("q4", t))
        check([a[7] for a in m], ex[t]["kx2"], ("|q(kx)|^2", t))
        check([a[16] for a in m], ex[t]["kd2"], ("|q(k_xy)|^2", t))


def test_replica_exchange_rate_L2():
    L, n_T, h = 2, 4, 0.3
    betas = W.geometric_betas(n_T, 0.5, 2.0)
    J = W.gaussian_couplings(9, 0, L)
    h32 = float(np.float32(h))
    E, ex = enumerate_L2(J, h32, betas)
    sts = run_independent(L, n_T, betas, h, W.J_GAUSS, J, runs=16, sweeps=1000, burn=10 ** 9,
                          mode=O.MODE_MIRROR)
    before = [st.swaps.copy() for st in sts]
    sweeps = 20000
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex_:
        list(ex_.map(lambda st: st.run(sweeps), sts))
    for t in range(n_T - 1):
        dB = betas[t] - betas[t + 1]
        A = np.minimum(1.0, np.exp(dB * (E[:, None] - E[None, :])))
        rate = ex[t]["pi"] @ A @ ex[t + 1]["pi"]
        attempts = sweeps // 2
        for r in range(2):
            check([(st.swaps[r, t] - b[r, t]) / attempts for st, b in zip(sts, before)], rate,
                  ("swap rate", r, t))


def test_equal_temperatures_always_swap():
    L, n_T = 2, 3
    betas = np.array([0.7, 0.7, 0.7])
    J = W.gaussian_couplings(3, 0, L)
    st = O.SampleState(L, n_T, betas, 0.2, W.J_GAUSS, J, W.initial_spins(3, 0, L, n_T), 3, 0)
    st.run(100)
    # pair t is attempted on the 50 sweeps with n = t mod 2
    assert (st.swaps[:, :2] == 50).all()


def test_zero_coupling_closed_forms():
    L, n_T, h = 4, 4, 0.3
    N = L ** 3
    betas = W.geometric_betas(n_T, 0.5, 2.0)
    J = np.zeros((3, N), dtype=np.float32)
    h32 = float(np.float32(h))
    sts = run_independent(L, n_T, betas, h, W.J_GAUSS, J, runs=12, sweeps=4000, burn=200,
                          mode=O.MODE_MIRROR)
    for t in range(n_T):
        m = math.tanh(betas[t] * h32)
        means = [st.acc[t] / st.acc[t, 0] for st in sts]
        check([a[32] for a in means], -h32 * N * m, ("E", t))
        check([a[1] for a in means], m * m, ("q", t))
        check([a[2] for a in means], 1.0 / N + (1.0 - 1.0 / N) * m ** 4, ("q2", t))
        # q(k) has zero mean and <|q(k)|^2> = (1 - m^4)/N for every k != 0
        check([a[5] for a in means], 0.0, ("Re q(kx)", t))
        check([a[7] for a in means], (1.0 - m ** 4) / N, ("|q(kx)|^2", t))
        check([a[7 + 3 * 4] for a in means], (1.0 - m ** 4) / N, ("|q(k_x-y)|^2", t))


@pytest.mark.parametrize("L,jkind", [(4, W.J_GAUSS), (6, W.J_PM1), (2, W.J_GAUSS)])
def test_incremental_energy_is_exact(L, jkind):
    n_T, h = 5, 0.25
    betas = W.geometric_betas(n_T, 0.6, 1.8)
    J = W.gaussian_couplings(2, 4, L) if jkind == W.J_GAUSS else W.pm1_couplings(2, 4, L)
    st = O.SampleState(L, n_T, betas, h, jkind, J, W.initial_spins(2, 4, L, n_T), 2, 4)
    for _ in range(3):
        st.run(70)
        for r in range(2):
            for w in range(n_T):
                EJ, M, _ = hamiltonian(L, J, st.spins[r, w], 0.0)
                assert st.EJ[r, w] == EJ
                assert st.M[r, w] == M
    # walker maps stay permutations
    for r in range(2):
        assert sorted(st.walker_at_slot[r]) == list(range(n_T))


def test_delta_e_matches_recomputed_energy():
    L, h = 4, 0.3
    h32 = float(np.float32(h))
    J = W.gaussian_couplings(8, 1, L)
    rng = np.random.default_rng(3)
    for _ in range(40):
        s = np.where(rng.random(L ** 3) < 0.5, 1, -1).astype(np.int8)
        i = int(rng.integers(L ** 3))
        s2 = s.copy()
        s2[i] = -s2[i]
        dE_exact = hamiltonian(L, J, s2, h32)[2] - hamiltonian(L, J, s, h32)[2]
        dE32 = O.delta_e32(L, W.J_GAUSS, J, s, h32, i)
        assert abs(dE32 - dE_exact) <= 2.0 * np.spacing(np.float32(abs(dE_exact)))


FAMILIES = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1),
            (0, 1, 1), (0, 1, -1)]


@pytest.mark.parametrize("L", [2, 4, 6])
def test_overlap_fourier_matches_fft(L):
    rng = np.random.default_rng(L)
    N = L ** 3
    sa = np.where(rng.random(N) < 0.6, 1, -1).astype(np.int8)
    sb = np.where(rng.random(N) < 0.3, 1, -1).astype(np.int8)
    acc, sums = O.measure_pair(L, sa, sb, Ea=-1.5, Eb=2.5)
    q = (sa.astype(np.float64) * sb).reshape(L, L, L)       # [z, y, x]
    F = np.fft.fftn(q)                                        # e^{-i k.r}
    q0 = q.sum() / N
    assert acc[0] == 1.0
    assert acc[1] == pytest.approx(q0, abs=1e-15)
    assert acc[4] == pytest.approx(q0 ** 4, abs=1e-15)
    for f, (kx, ky, kz) in enumerate(FAMILIES):
        v = np.conj(F[kz % L, ky % L, kx % L]) / N            # e^{+i k.r}
        assert acc[5 + 3 * f] == pytest.approx(v.real, abs=1e-13), f
        assert acc[6 + 3 * f] == pytest.approx(v.imag, abs=1e-13), f
        assert acc[7 + 3 * f] == pytest.approx(abs(v) ** 2, abs=1e-13), f
    assert (acc[32], acc[33], acc[34], acc[35]) == (-1.5, 2.25, 2.5, 6.25)


def test_overlap_hand_configurations():
    L = 4
    N = L ** 3
    up = np.ones(N, dtype=np.int8)
    acc, _ = O.measure_pair(L, up, -up)
    assert acc[1] == -1.0 and acc[2] == 1.0
    assert np.allclose(acc[5:32], 0.0, atol=1e-15)
    # q_i = +1 for x < L/2, -1 otherwise: Re q(k_x) = (1/L) sum_c sign_c cos(2 pi c/L)
    x = np.arange(N) % L
    sb = np.where(x < L // 2, 1, -1).astype(np.int8)
    acc, _ = O.measure_pair(L, up, sb)
    expect = sum((1 if c < L // 2 else -1) * math.cos(2 * math.pi * c / L) for c in range(L)) / L
    assert acc[5] == pytest.approx(expect, abs=1e-15)
    assert acc[8] == pytest.approx(0.0, abs=1e-15)     # k along y sees a constant field


def test_sample_independence_and_reproducibility():
    work = W.config_workload("L4_gauss", samples=[3, 7], measure_start=10)
    a = O.OracleEnsemble(work).run(60)
    b = O.OracleEnsemble(work.subset([1])).run(60)
    assert np.array_equal(a.states[1].spins, b.states[0].spins)
    assert np.array_equal(a.states[1].acc, b.states[0].acc)
    c = O.OracleEnsemble(work).run(25)
    c.run(35)
    for x, y in zip(a.states, c.states):
        assert np.array_equal(x.spins, y.spins)
        assert np.array_equal(x.acc, y.acc)
        assert np.array_equal(x.walker_at_slot, y.walker_at_slot)
