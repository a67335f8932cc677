"""Pins of the oracle's finalize step (eqs. 3-6, jackknife) against closed forms.

With zero couplings the overlaps q_i are independent +-1 variables with mean
mu = m^2, so q = (2K - N)/N with K ~ Binomial(N, (1 + mu)/2).  Raw moments of q
computed from the binomial law give accumulators whose observables have closed
forms:  chi(0) = chi(k) = 1 - mu^2,  g = (1 - 3 mu^2) / (N (1 - mu^2)),
xi_L = 0, R12 = 1.  At zero field (mu = 0, odd moments vanish) eq. 3 reduces to
g = (3 - <q^4>/<q^2>^2)/2.  The jackknife error of a disorder mean equals the
standard error of the mean.
"""
import math
from fractions import Fraction
from math import comb

import numpy as np
import pytest

from oracle import ea_oracle as O


def binomial_moments(N, mu):
    """Exact raw moments of q = (2K - N)/N, K ~ Binomial(N, (1 + mu)/2), as
    rationals, rounded once to binary64."""
    mu = Fraction(mu).limit_denominator(10 ** 6)
    p = (1 + mu) / 2
    out = []
    for j in range(1, 5):
        v = sum(comb(N, k) * p ** k * (1 - p) ** (N - k) * Fraction(2 * k - N, N) ** j
                for k in range(N + 1))
        out.append(float(v))
    return out


def synthetic_acc(L, mus, n=1000.0):
    """[1][n_T][36] accumulators whose thermal means are the exact J = 0 values."""
    N = L ** 3
    acc = np.zeros((1, len(mus), O.NACC))
    for t, mu in enumerate(mus):
        q1, q2, q3, q4 = binomial_moments(N, mu)
        acc[0, t, 0] = n
        acc[0, t, 1:5] = n * np.array([q1, q2, q3, q4])
        for f in range(O.NPLANE):
            acc[0, t, 7 + 3 * f] = n * (1.0 - mu * mu) / N   # <|q(k)|^2>, <q(k)> = 0
    return acc


@pytest.mark.parametrize("L", [4, 6, 8])
def test_zero_coupling_observables(L):
    N = L ** 3
    mus = [0.05, 0.3, 0.5]
    mus = [float(Fraction(m).limit_denominator(10 ** 6)) for m in mus]
    obs = O.observables(synthetic_acc(L, mus), L)
    for t, mu in enumerate(mus):
        assert obs["chi0"][t] == pytest.approx(1.0 - mu * mu, rel=1e-10)
        assert obs["chi_kmin"][t] == pytest.approx(1.0 - mu * mu, rel=1e-10)
        assert obs["chi_k2"][t] == pytest.approx(1.0 - mu * mu, rel=1e-10)
        g_exact = (1 - 3 * mu * mu) / (N * (1 - mu * mu))
        # eq. 3 centres on the disorder mean; the raw-moment expansion cancels
        # ~1e4 eps at N = 512 and g is ~1e-3 of the 3 it is taken from
        assert obs["g"][t] == pytest.approx(g_exact, rel=1e-6)
        assert obs["R12"][t] == pytest.approx(1.0, rel=1e-10)
        assert obs["chi0_over_chikmin"][t] == pytest.approx(1.0, rel=1e-10)


def test_zero_field_binder_reduction():
    rng = np.random.default_rng(1)
    S, nT, L = 7, 3, 6
    acc = np.zeros((S, nT, O.NACC))
    acc[..., 0] = 100.0
    acc[..., 2] = 100.0 * rng.uniform(0.2, 0.4, size=(S, nT))
    acc[..., 4] = 100.0 * rng.uniform(0.1, 0.2, size=(S, nT))
    obs = O.observables(acc, L)
    q2 = (acc[..., 2] / 100.0).mean(axis=0)
    q4 = (acc[..., 4] / 100.0).mean(axis=0)
    assert np.allclose(obs["g"], 0.5 * (3.0 - q4 / q2 ** 2), rtol=1e-13)


def test_correlation_length_of_ornstein_zernike_ratio():
    # chi(0)/chi(kmin) = 1 + (2 sin(pi/L) xi)^2 must give back xi  (eq. 5)
    L, N, xi = 8, 512, 1.7
    acc = np.zeros((1, 1, O.NACC))
    acc[0, 0, 0] = 1.0
    acc[0, 0, 2] = 4.0 / N                                  # chi(0) = 4
    chik = 4.0 / (1.0 + (2.0 * math.sin(math.pi / L) * xi) ** 2)
    for f in range(3):
        acc[0, 0, 7 + 3 * f] = chik / N
    obs = O.observables(acc, L)
    assert obs["xi_L"][0] == pytest.approx(xi, rel=1e-12)


def test_jackknife_of_mean_is_standard_error():
    rng = np.random.default_rng(2)
    S, L = 9, 4
    acc = np.zeros((S, 2, O.NACC))
    acc[..., 0] = 10.0
    acc[..., 1] = 10.0 * rng.normal(0.3, 0.05, size=(S, 2))
    acc[..., 2] = 1.0
    jk = O.jackknife(acc, L)
    val, err = jk["q"]
    per = acc[..., 1] / 10.0
    assert np.allclose(val, per.mean(axis=0), rtol=1e-14)
    assert np.allclose(err, per.std(axis=0, ddof=1) / math.sqrt(S), rtol=1e-12)


# --------------------------------------------------------------------------
# The disorder average is read as the exact sum rounded once (then one
# rounded division by the count).  Pinned against math.fsum (a correctly
# rounded library sum) and exact rationals, on inputs chosen to defeat
# ordinary summation: cancellation, exponents far apart, subnormals.
def adversarial_arrays():
    rng = np.random.default_rng(7)
    yield np.array([1e16, 1.0, -1e16, 1e-16, 3.0])
    yield np.array([2.0 ** 53, 1.0, 1.0, -2.0 ** 53])          # ties broken by the tail
    yield np.array([1.0, 2.0 ** -53, 2.0 ** -106])             # half-way plus a sticky bit
    yield np.array([1.0, -2.0 ** -54, 2.0 ** -107])
    yield np.array([5e-324, 5e-324, -1e-320, 2.2250738585072014e-308])
    yield np.array([1e300, -1e300, 1e-300, 7.0])
    yield rng.normal(size=257) * 10.0 ** rng.integers(-30, 30, size=257)
    v = rng.normal(size=100)
    yield np.concatenate([v, -v, [1e-17]])                     # exact cancellation but a tail
    yield rng.uniform(0.0, 1.0, size=2048)                    # the shape of real disorder sums


def test_exact_sum_matches_fsum_and_rationals():
    for a in adversarial_arrays():
        ref = math.fsum(a.tolist())
        assert O.exact_sum(a) == ref
        exact = sum(Fraction(x) for x in a.tolist())
        assert O.exact_sum(a) == float(exact)
        perm = np.random.default_rng(3).permutation(a)
        assert O.exact_sum(perm) == ref


def test_leave_one_out_matches_fsum():
    for a in adversarial_arrays():
        col = O.ExactColumn(a)
        idx = range(len(a)) if len(a) < 40 else range(0, len(a), 37)
        for s in idx:
            assert col.rounded_without(s) == math.fsum(np.delete(a, s).tolist()), s


def test_exact_sum_non_finite():
    assert math.isnan(O.exact_sum([1.0, math.nan, 2.0]))
    assert math.isnan(O.exact_sum([math.inf, -math.inf]))
    assert O.exact_sum([math.inf, 1.0, 1e308]) == math.inf
    assert O.exact_sum([-math.inf, 1.0]) == -math.inf
    col = O.ExactColumn([1.0, math.nan, 2.5])
    assert col.rounded_without(1) == 3.5 and math.isnan(col.rounded_without(0))


def test_disorder_mean_is_rounded_exact_sum_over_count():
    rng = np.random.default_rng(5)
    S, nT = 13, 3
    acc = np.zeros((S, nT, O.NACC))
    acc[..., 0] = rng.integers(1, 50, size=(S, nT)).astype(np.float64)
    acc[..., 1:] = rng.normal(size=(S, nT, O.NACC - 1)) * acc[..., 0:1]
    D = O.disorder_means(acc)
    for t in range(nT):
        for j in range(O.NACC):
            m = [acc[s, t, j] / acc[s, t, 0] for s in range(S)]
            assert D[t, j] == math.fsum(m) / S


def test_observables_do_not_depend_on_sample_order():
    rng = np.random.default_rng(9)
    S, nT, L = 40, 4, 6
    acc = np.zeros((S, nT, O.NACC))
    acc[..., 0] = 100.0
    acc[..., 1:] = rng.uniform(0.0, 1.0, size=(S, nT, O.NACC - 1)) * 100.0
    perm = rng.permutation(S)
    a, b = O.jackknife(acc, L), O.jackknife(acc[perm], L)
    for k in a:
        assert np.array_equal(a[k][0], b[k][0], equal_nan=True), k
        assert np.array_equal(a[k][1], b[k][1], equal_nan=True), k
