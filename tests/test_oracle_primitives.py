"""Pins of the oracle's primitives against published values and mathematics.

* Philox4x32-10 against the generator's published known-answer vectors.
* exp_ea32 / exp_ea64 against the exponential itself: binary64 libm on a dense
  sweep of every 101st binary32 input in [-86, 0], and a 40-digit decimal
  exponential for binary64 inputs (error bounds, special cases).
"""
import os
import struct
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import ea_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert O.philox4x32_10(ctr, key) == expect


def test_philox_counter_sensitivity():
    # every counter and key word reaches every output word (no dropped input)
    base = O.philox4x32_10([1, 2, 3, 4], [5, 6])
    for pos in range(6):
        c, k = [1, 2, 3, 4], [5, 6]
        if pos < 4:
            c[pos] ^= 1
        else:
            k[pos - 4] ^= 1
        out = O.philox4x32_10(c, k)
        assert all(a != b for a, b in zip(out, base)), pos


def _f32_grid(step):
    lo = 0x80000000                                          # -0.0
    hi = struct.unpack("<I", struct.pack("<f", -86.0))[0]     # -86.0
    bits = np.arange(lo, hi + 1, step, dtype=np.uint64).astype(np.uint32)
    return bits.view(np.float32)


def test_exp_ea32_accuracy_dense():
    x = _f32_grid(101)
    y = O.exp_ea32_n(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    err = np.abs(y - ref) / ulp
    assert err.max() <= 1.5, err.max()
    # monotone non-increasing as x decreases (the sweep of x is descending)
    assert np.all(np.diff(y) <= 0.0)


def test_exp_ea32_special_values():
    assert O.exp_ea32(0.0) == 1.0
    assert O.exp_ea32(-0.0) == 1.0
    assert O.exp_ea32(-86.0) > 0.0
    assert O.exp_ea32(np.nextafter(np.float32(-86.0), np.float32(-100.0))) == 0.0
    assert O.exp_ea32(-1000.0) == 0.0
    # results never fall below the smallest normal binary32
    assert O.exp_ea32(-86.0) >= np.finfo(np.float32).tiny


def test_exp_ea64_accuracy_decimal():
    getcontext().prec = 40
    rng = np.random.default_rng(7)
    xs = np.concatenate([-rng.random(400) * 700.0, -rng.random(200) * 2.0, -rng.random(100) * 1e-6])
    y = O.exp_ea64_n(xs)
    for x, v in zip(xs, y):
        exact = Decimal(float(x)).exp()
        ulp = np.spacing(float(exact))
        assert abs(Decimal(float(v)) - exact) <= Decimal(ulp) * Decimal("1.0"), x


def test_exp_ea64_special_values():
    assert O.exp_ea64(0.0) == 1.0
    assert O.exp_ea64(-700.0) > 0.0
    assert O.exp_ea64(-700.0000001) == 0.0


def test_exchange_shortcut_bounds():
    # The kernels' exchange test (u53 < exp_ea64(D), D < 0) rejects outright
    # below D = -40 and otherwise compares u53 with the hardware 2^y,
    # y = fl32(D log2 e), widened by a relative 2^-16.  The bounds it rests on:
    # exp_ea64 below -40 is under the smallest positive 53-bit uniform ...
    assert O.exp_ea64(-40.0) < 2.0 ** -57 < 2.0 ** -53
    xs = -40.0 - np.random.default_rng(3).random(1000) * 700.0
    assert (O.exp_ea64_n(xs) < 2.0 ** -57).all()
    # ... rounding D log2 e (|.| < 58) to binary32 moves y by at most 2^-19 ...
    rng = np.random.default_rng(4)
    D = -rng.random(100000) * 40.0
    t = D * 1.4426950408889634
    y = t.astype(np.float32).astype(np.float64)
    assert np.abs(y - t).max() <= 2.0 ** -19
    # ... so with the hardware exponential within 2^-22 of 2^y (checked on every
    # binary32 by ea_verify_exchange_bracket) and exp_ea64 within 2^-49 of e^D,
    # the estimate stays well inside the margin
    assert (2.0 ** (2.0 ** -19) - 1.0) * 1.0001 + 2.0 ** -22 + 2.0 ** -49 < 1.7e-6 < 2.0 ** -16
