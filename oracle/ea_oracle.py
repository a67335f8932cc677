"""Python face of the CPU oracle (``ea_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; both consume the same seeded input arrays.

The oracle follows arXiv:1403.4560 (Methods: eq. 1 Hamiltonian, parallel
tempering with two replicas per temperature, eqs. 2-6 observables) under the
numeric contract stated in the header of ``ea_oracle.c``.  The finalize step
(disorder averages, eqs. 3-6, jackknife over samples) is written here in plain
numpy, one formula per observable.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ea_oracle.c")
_LIB = os.path.join(_HERE, "libea_oracle.so")

NACC = 36      # accumulators per (sample, slot)
NPLANE = 9     # plane-sum families (3 axes, 6 diagonals)
J_GAUSS, J_PM1 = 0, 1
MODE_MIRROR, MODE_FP64 = 0, 1

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.POINTER
        L.eao_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.eao_exp_ea32.argtypes = [ctypes.c_float]
        L.eao_exp_ea32.restype = ctypes.c_float
        L.eao_exp_ea64.argtypes = [ctypes.c_double]
        L.eao_exp_ea64.restype = ctypes.c_double
        L.eao_energy.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 P(ctypes.c_double), P(ctypes.c_int32)]
        L.eao_delta_e32.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_float, ctypes.c_int32]
        L.eao_delta_e32.restype = ctypes.c_float
        L.eao_pm1_thresholds.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]
        L.eao_measure_pair.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.eao_run.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_float, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int64,
            ctypes.c_int32, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p]
        L.eao_run.restype = ctypes.c_int
        L.eao_exp_ea32_n.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.eao_exp_ea64_n.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# primitives
def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().eao_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def exp_ea32(x: float) -> float:
    return float(lib().eao_exp_ea32(float(np.float32(x))))


def exp_ea64(x: float) -> float:
    return float(lib().eao_exp_ea64(float(x)))


def exp_ea32_n(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().eao_exp_ea32_n(_ptr(x), _ptr(y), x.size)
    return y


def exp_ea64_n(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().eao_exp_ea64_n(_ptr(x), _ptr(y), x.size)
    return y


def energy(L: int, jkind: int, J: np.ndarray, s: np.ndarray):
    """Exact (E_J, M) of one configuration: E = E_J - h M (eq. 1)."""
    J = np.ascontiguousarray(J)
    s = np.ascontiguousarray(s, dtype=np.int8)
    e = ctypes.c_double()
    m = ctypes.c_int32()
    lib().eao_energy(L, jkind, _ptr(J), _ptr(s), ctypes.byref(e), ctypes.byref(m))
    return e.value, m.value


def delta_e32(L, jkind, J, s, h32, i):
    J = np.ascontiguousarray(J)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(lib().eao_delta_e32(L, jkind, _ptr(J), _ptr(s), float(np.float32(h32)), int(i)))


def pm1_thresholds(beta: np.ndarray, h32: float) -> np.ndarray:
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.zeros((len(beta), 2, 7), dtype=np.uint32)
    lib().eao_pm1_thresholds(len(beta), _ptr(beta), float(np.float32(h32)), _ptr(out))
    return out


def measure_pair(L, sa, sb, Ea=0.0, Eb=0.0):
    sa = np.ascontiguousarray(sa, dtype=np.int8)
    sb = np.ascontiguousarray(sb, dtype=np.int8)
    acc = np.zeros(NACC, dtype=np.float64)
    sums = np.zeros(1 + NPLANE * L, dtype=np.int32)
    lib().eao_measure_pair(L, _ptr(sa), _ptr(sb), float(Ea), float(Eb), _ptr(acc), _ptr(sums))
    return acc, sums


# --------------------------------------------------------------------------
# one disorder sample
class SampleState:
    """Full state of one disorder sample (both chains, all slots)."""

    def __init__(self, L, n_T, beta, h32, jkind, J, spins0, seed, sample_id,
                 measure_every=0, measure_start=0, mode=MODE_MIRROR, trace_cap=0):
        self.L, self.n_T = int(L), int(n_T)
        self.N = self.L ** 3
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        self.h32 = float(np.float32(h32))
        self.jkind = int(jkind)
        self.J = np.ascontiguousarray(J).reshape(3, self.N)
        self.seed, self.sample_id = int(seed), int(sample_id)
        self.measure_every, self.measure_start = int(measure_every), int(measure_start)
        self.mode = int(mode)
        self.spins = np.array(spins0, dtype=np.int8).reshape(2, self.n_T, self.N).copy()
        self.walker_at_slot = np.tile(np.arange(self.n_T, dtype=np.int32), (2, 1))
        self.EJ = np.zeros((2, self.n_T), dtype=np.float64)
        self.M = np.zeros((2, self.n_T), dtype=np.int32)
        for r in range(2):
            for w in range(self.n_T):
                self.EJ[r, w], self.M[r, w] = energy(self.L, self.jkind, self.J, self.spins[r, w])
        self.sweep = np.zeros(1, dtype=np.int64)
        self.acc = np.zeros((self.n_T, NACC), dtype=np.float64)
        self.flips = np.zeros((2, self.n_T), dtype=np.int64)
        self.swaps = np.zeros((2, self.n_T), dtype=np.int64)
        self.trace_cap = int(trace_cap)
        self.trace = np.zeros((max(self.trace_cap, 1), self.n_T, 1 + NPLANE * self.L), dtype=np.int32)
        self.trace_len = np.zeros(1, dtype=np.int64)

    def run(self, n_sweeps: int):
        rc = lib().eao_run(
            self.L, self.n_T, _ptr(self.beta), self.h32, self.jkind, _ptr(self.J),
            ctypes.c_uint64(self.seed), ctypes.c_uint32(self.sample_id), self.measure_every,
            self.measure_start, self.mode, int(n_sweeps),
            _ptr(self.spins), _ptr(self.walker_at_slot), _ptr(self.EJ), _ptr(self.M),
            _ptr(self.sweep), _ptr(self.acc), _ptr(self.flips), _ptr(self.swaps),
            _ptr(self.trace) if self.trace_cap > 0 else None, self.trace_cap,
            _ptr(self.trace_len))
        if rc != 0:
            raise ValueError("oracle rejected the sample parameters")
        return self

    def energies(self) -> np.ndarray:
        """E = E_J - h M per (chain, walker), binary64."""
        return self.EJ - np.float64(self.h32) * self.M.astype(np.float64)

    def spins_slot_order(self) -> np.ndarray:
        out = np.empty_like(self.spins)
        for r in range(2):
            out[r] = self.spins[r, self.walker_at_slot[r]]
        return out

    def energies_slot_order(self) -> np.ndarray:
        E = self.energies()
        return np.stack([E[r, self.walker_at_slot[r]] for r in range(2)])


class OracleEnsemble:
    """A batch of independent samples, run on host threads (one per sample at a
    time).  ``work`` is a ``paper_1403_4560_amd.workload.Workload``-shaped
    object exposing per-sample arrays."""

    def __init__(self, work, samples=None, mode=MODE_MIRROR, trace_cap=0):
        self.idx = list(range(work.n_samples)) if samples is None else list(samples)
        self.states = []
        for s in self.idx:
            self.states.append(SampleState(
                work.L[s], work.n_temps[s], work.beta_of(s), work.h[s], work.jkind,
                work.J_of(s), work.spins0_of(s), work.seed, work.sample_id[s],
                work.measure_every, work.measure_start, mode, trace_cap))

    def run(self, n_sweeps: int, threads: int | None = None):
        threads = threads or min(len(self.states), os.cpu_count() or 1)
        if threads <= 1:
            for st in self.states:
                st.run(n_sweeps)
        else:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(lambda st: st.run(n_sweeps), self.states))
        return self


# --------------------------------------------------------------------------
# finalize: disorder averages (overline) of thermal averages (<...>), eqs. 3-6
#
# Reading of the disorder average (the paper's overline, an average over
# disorder realizations of one model at one field and ladder): the exact sum
# of the S per-sample values, rounded once to binary64 (nearest, ties to even),
# then divided by S in one rounded division.  A leave-one-sample-out replicate
# (jackknife) is the exact sum of the other S - 1 values rounded once, divided
# by S - 1.  Exact sums are integer sums in units of 2^-1074 (every finite
# binary64 is an integer multiple of that unit), so no result depends on the
# order of the samples.  Non-finite values follow IEEE addition: any NaN, or
# +inf together with -inf, gives NaN; otherwise an infinity wins.
_UNIT_EXP = 1074


def _as_units(x: float) -> int:
    """Finite binary64 x as the exact integer x * 2^1074."""
    n, d = float(x).as_integer_ratio()
    return n << (_UNIT_EXP - (d.bit_length() - 1))


def _from_units(v: int) -> float:
    """v * 2^-1074 rounded once to binary64 (int true division is correctly
    rounded)."""
    try:
        return v / (1 << _UNIT_EXP)
    except OverflowError:
        return math.copysign(math.inf, v)


class ExactColumn:
    """The exact sum of a multiset of binary64 values (one column: one slot
    and one accumulator, over samples)."""

    def __init__(self, values):
        v = np.asarray(values, dtype=np.float64)
        fin = np.isfinite(v)
        self.n_nan = int(np.isnan(v).sum())
        self.n_pinf = int((v == np.inf).sum())
        self.n_ninf = int((v == -np.inf).sum())
        self.units = [(_as_units(x) if ok else 0) for x, ok in zip(v.tolist(), fin.tolist())]
        self.total = sum(self.units)
        self.values = v

    def _special(self, n_nan, n_pinf, n_ninf):
        if n_nan or (n_pinf and n_ninf):
            return math.nan
        if n_pinf:
            return math.inf
        if n_ninf:
            return -math.inf
        return None

    def rounded(self) -> float:
        """The correctly rounded sum of every value."""
        sp = self._special(self.n_nan, self.n_pinf, self.n_ninf)
        return sp if sp is not None else _from_units(self.total)

    def rounded_without(self, s: int) -> float:
        """The correctly rounded sum of every value but the s-th."""
        x = float(self.values[s])
        sp = self._special(self.n_nan - math.isnan(x), self.n_pinf - (x == math.inf),
                           self.n_ninf - (x == -math.inf))
        return sp if sp is not None else _from_units(self.total - self.units[s])


def exact_sum(values) -> float:
    """Correctly rounded sum of binary64 values (equals math.fsum on finite
    input)."""
    return ExactColumn(values).rounded()


def thermal_means(acc: np.ndarray) -> np.ndarray:
    """Per-sample thermal averages <.> = accumulated sum / number of
    measurements; acc has shape [S][n_T][36]."""
    n = acc[..., 0:1]
    with np.errstate(invalid="ignore", divide="ignore"):
        return acc / n


OBS_NAMES = ("q", "chi0", "chi_kmin", "chi_k2", "g", "xi_L", "R12", "chi0_over_chikmin", "E_a", "E_b")


def observables_of_means(D: np.ndarray, L: int) -> dict:
    """Observables per temperature slot from disorder-averaged thermal means
    D [n_T][36] (column layout of the accumulators), each formula evaluated
    in the order written (binary64, one rounding per operation):

    chi(k) = N([<|q(k)|^2>] - |[<q(k)>]|^2)                          eq. 4
    chi(k_min) = (chi_x + chi_y + chi_z) / 3                     Results
    chi(k2) = mean of the six (1,1,0) images, summed in image order
    g = (3 - [<(q-Q)^4>] / [<(q-Q)^2>]^2) / 2, Q = [<q(0)>], the central
        moments expanded in raw moments                               eq. 3
    xi_L = sqrt(chi(0)/chi(k_min) - 1) / (2 sin(pi/L))                eq. 5
    R12 = chi(k_min) / chi(k2)                                        eq. 6
    """
    N = float(L * L * L)
    D = np.asarray(D, dtype=np.float64)
    q1, q2, q3, q4 = D[:, 1], D[:, 2], D[:, 3], D[:, 4]
    Q = q1
    c2 = q2 - 2.0 * Q * q1 + Q * Q
    c4 = q4 - 4.0 * Q * q3 + 6.0 * Q * Q * q2 - 4.0 * Q * Q * Q * q1 + Q * Q * Q * Q
    chi = []
    for f in range(NPLANE):
        re, im, k2 = D[:, 5 + 3 * f], D[:, 6 + 3 * f], D[:, 7 + 3 * f]
        chi.append(N * (k2 - (re * re + im * im)))
    chi0 = N * (q2 - q1 * q1)
    chi_kmin = (chi[0] + chi[1] + chi[2]) / 3.0
    chi_k2 = (chi[3] + chi[4] + chi[5] + chi[6] + chi[7] + chi[8]) / 6.0
    with np.errstate(invalid="ignore", divide="ignore"):
        g = 0.5 * (3.0 - c4 / (c2 * c2))
        xi = np.sqrt(chi0 / chi_kmin - 1.0) / (2.0 * math.sin(math.pi / L))
        r12 = chi_kmin / chi_k2
        ratio = chi0 / chi_kmin
    return {"q": q1, "chi0": chi0, "chi_kmin": chi_kmin, "chi_k2": chi_k2, "g": g, "xi_L": xi,
            "R12": r12, "chi0_over_chikmin": ratio, "E_a": D[:, 32], "E_b": D[:, 34]}


def _columns(m: np.ndarray):
    """ExactColumn per (slot, accumulator) of per-sample values m [S][n_T][K]."""
    return [[ExactColumn(m[:, t, j]) for j in range(m.shape[2])] for t in range(m.shape[1])]


def disorder_means(acc: np.ndarray) -> np.ndarray:
    """[n_T][36] disorder averages of the thermal means of S samples of one
    system (the reading above)."""
    m = thermal_means(np.asarray(acc, dtype=np.float64))
    S = m.shape[0]
    cols = _columns(m)
    return np.array([[c.rounded() / S for c in row] for row in cols])


def observables(acc: np.ndarray, L: int) -> dict:
    """Disorder-averaged observables per temperature slot from the
    accumulators of S samples of one system ([S][n_T][36])."""
    out = observables_of_means(disorder_means(acc), L)
    out["xi_over_L"] = out["xi_L"] / L
    return out


def jackknife(acc: np.ndarray, L: int) -> dict:
    """Leave-one-sample-out jackknife errors of every observable (Methods,
    last paragraph: statistical errors from disorder averaging).  Replicate
    s: observables of the means of the other S - 1 samples; mean of the
    replicates theta_bar = (exact sum)/S; error sqrt(((S-1)/S) sum_s
    (theta_s - theta_bar)^2) with the sum exact and rounded once."""
    m = thermal_means(np.asarray(acc, dtype=np.float64))
    S, nT = m.shape[0], m.shape[1]
    full = observables(acc, L)
    if S < 2:
        return {k: (v, np.full_like(v, np.nan)) for k, v in full.items()}
    cols = _columns(m)
    reps = []
    for s in range(S):
        Ds = np.array([[c.rounded_without(s) / (S - 1) for c in row] for row in cols])
        reps.append(observables_of_means(Ds, L))
    out = {}
    for k in OBS_NAMES:
        R = np.stack([r[k] for r in reps])                  # [S][n_T]
        err = np.empty(nT)
        for t in range(nT):
            bar = exact_sum(R[:, t]) / S
            d = R[:, t] - bar
            err[t] = math.sqrt((S - 1) / S * exact_sum(d * d))
        out[k] = (full[k], err)
    out["xi_over_L"] = (full["xi_over_L"], out["xi_L"][1] / L)
    return out
