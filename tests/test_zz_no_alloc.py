"""GPU: the no-allocation jackknife (ea_finalize_jackknife_noalloc) against
ea_finalize_jackknife, through the C ABI.

The variant keeps its replicate scratch in a fixed per-device array instead of
memory the library allocates; its results must be bit-identical to the
allocating entry point's, on two calls in a row (the second with a smaller
selection, so stale scratch from the first call would show), and it must
refuse a selection beyond its fixed size.
"""
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


def same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k][0], b[k][0], equal_nan=True), (k, "value")
        assert np.array_equal(a[k][1], b[k][1], equal_nan=True), (k, "error")


def test_noalloc_jackknife_matches_allocating_entry_point(torch_cuda):
    from paper_1403_4560_amd import binding
    work = W.config_workload("L8_gauss", samples=range(24), measure_start=0)
    print("case: no-allocation jackknife, L8 24 samples", flush=True)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(60)
        acc = np.stack(ens.measure()["acc"])
        first = ens.finalize_jackknife(noalloc=True)           # all 24 samples
        ref_first = ens.finalize_jackknife()
        sub = [3, 17, 5, 22, 9]
        second = ens.finalize_jackknife(sub, noalloc=True)     # smaller: 5 samples
        ref_second = ens.finalize_jackknife(sub)
    same(first, ref_first)
    same(second, ref_second)
    rjk = O.jackknife(acc, 8)
    for k in O.OBS_NAMES:
        assert np.array_equal(first[k][0], rjk[k][0], equal_nan=True), k
        assert np.array_equal(first[k][1], rjk[k][1], equal_nan=True), k


def test_noalloc_jackknife_refuses_selections_beyond_its_scratch(torch_cuda):
    from paper_1403_4560_amd import binding
    # 64 slots x 1700 samples = 108800 replicates > 104857
    work = W.make_workload([4] * 1700, 64, (0.5, 2.0), 0.3, name="too many replicates")
    print("case: no-allocation jackknife beyond its scratch", flush=True)
    with binding.Ensemble(work) as ens:
        ens.sweep_pt(20)
        with pytest.raises(binding.EAError) as err:
            ens.finalize_jackknife(noalloc=True)
        assert err.value.status == -1
        ok = ens.finalize_jackknife(list(range(1638)), noalloc=True)   # 64 x 1638 = 104832 fits
        ref = ens.finalize_jackknife(list(range(1638)))
    same(ok, ref)
