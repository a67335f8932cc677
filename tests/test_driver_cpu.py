"""Host logic of the Table I driver: bin schedule, exchange bookkeeping,
binning test and the Table I workload shape (no GPU)."""
import math

import numpy as np
import pytest

from paper_1403_4560_amd import driver as D


def test_table1_workload_shape():
    work = D.table1_workload(10, 3, first_sample=7)
    assert work.n_samples == 3 and list(work.sample_id) == [7, 8, 9]
    assert all(int(n) == 56 for n in work.n_temps) and all(int(L) == 10 for L in work.L)
    b = work.beta_of(0)
    assert b[0] == 0.1 and math.isclose(b[-1], 1.8, rel_tol=1e-14)
    ratios = b[1:] / b[:-1]
    assert np.allclose(ratios, ratios[0], rtol=1e-13)          # geometric (Table I caption)
    assert np.all(work.h == np.float32(0.1)) and work.jkind == 1
    assert set(np.unique(work.J_of(0))) <= {-1, 1}


@pytest.mark.parametrize("m,k", [(1, 1), (2, 2), (10, 4), (16, 5)])
def test_first_bin_holds_two_measurements(m, k):
    assert D.first_bin_for(m) == k
    lo, hi = 2 ** k, 2 ** (k + 1)
    assert hi // m - lo // m >= 2
    assert (hi // 2) // m - (lo // 2) // m < 2


def test_exchange_attempts_match_the_schedule():
    for lo, hi in [(16, 32), (1, 2), (3, 10), (0, 7)]:
        for t in range(5):
            brute = sum(1 for n in range(lo, hi) if n % 2 == t % 2)
            assert D.exchange_attempts(lo, hi, t) == brute


def _bin(k, v, e):
    return D.Bin(k, 2 ** k, 2 ** (k + 1), 1, {"R12": (np.array([0.0, v]), np.array([0.0, e]))},
                 np.zeros(1), np.zeros(2))


def test_binning_test_decision():
    ok = [_bin(4, 1.00, 0.05), _bin(5, 1.02, 0.03), _bin(6, 1.01, 0.02)]
    assert D.bins_agree(ok)
    drifting = [_bin(4, 0.80, 0.02), _bin(5, 0.95, 0.02), _bin(6, 1.01, 0.02)]
    assert not D.bins_agree(drifting)
    assert not D.bins_agree(ok[:2])                                  # fewer than three bins
    assert not D.bins_agree([_bin(4, float("nan"), 0.1)] + ok[1:])
