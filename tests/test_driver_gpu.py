"""GPU: the Table I driver's log-binned accumulators and the device jackknife
against the oracle, bin by bin."""
import numpy as np
import pytest

from oracle import ea_oracle as O
from paper_1403_4560_amd import driver as D

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def oracle_bins(work, log2_sweeps, k0):
    ens = O.OracleEnsemble(work)
    ens.run(2 ** k0)
    out = []
    for k in range(k0, log2_sweeps):
        for st in ens.states:
            st.acc[:] = 0.0
            st.flips[:] = 0
            st.swaps[:] = 0
        ens.run(2 ** k)
        out.append(np.stack([st.acc for st in ens.states]))
    return out


@pytest.mark.parametrize("L,samples", [(6, 4), (8, 3)])
def test_driver_bins_match_oracle(torch_cuda, L, samples):
    work = D.table1_workload(L, samples, first_sample=11)
    k0, K = D.first_bin_for(work.measure_every), 7
    print("case: driver L=%d S=%d bins %d..%d" % (L, samples, k0, K - 1), flush=True)
    from paper_1403_4560_amd import binding
    seen = []

    # the driver's own run, with each bin's accumulators captured
    orig = binding.Ensemble.finalize_jackknife

    def spy(self, *a, **k):
        seen.append(np.stack(self.measure()["acc"]))
        return orig(self, *a, **k)

    binding.Ensemble.finalize_jackknife = spy
    try:
        bins = D.run_log_binned(work, K)
    finally:
        binding.Ensemble.finalize_jackknife = orig
    ref = oracle_bins(work, K, k0)
    assert [b.k for b in bins] == list(range(k0, K)) and len(seen) == len(ref)
    for b, acc_gpu, acc_ref in zip(bins, seen, ref):
        assert np.array_equal(acc_gpu, acc_ref), ("bin", b.k)
        assert b.measurements == int(acc_ref[0, 0, 0])
        jk = O.jackknife(acc_ref, L)
        for name, (v, e) in b.obs.items():
            if name == "n_samples":
                assert np.all(v == samples)
                continue
            rv, re_ = jk[name]
            assert np.array_equal(v, rv, equal_nan=True), (b.k, name, v, rv)
            assert np.array_equal(e, re_, equal_nan=True), (b.k, name, "error", e, re_)
        assert np.all((b.flip_rate > 0) & (b.flip_rate < 1))
        assert np.all((b.swap_rate >= 0) & (b.swap_rate <= 1))
