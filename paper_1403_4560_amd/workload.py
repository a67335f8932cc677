"""Seeded synthetic inputs: disorder samples, temperature ladders and initial
spins.  This module holds none of the simulation's arithmetic; it only draws
the input arrays that the GPU library and the CPU oracle both consume.

Recipe (shapes follow the paper's workloads, Methods and Table I):
  * couplings per sample ``s``: numpy PCG64 stream seeded with
    SeedSequence([seed, sample_id, 2]).
      - Gaussian (zero mean, unit variance, Methods/Conclusion): a normal
        deviate rounded to the nearest multiple of 2^-18 and clamped to
        |J| <= (2^21 - 1) 2^-18, stored as float32 (exact);
      - bimodal +-1 with probability 1/2 each (Methods), stored as int8.
    Layout [3][N]: bond d of site i joins i and i + d (d = x, y, z).
  * initial spins: SeedSequence([seed, sample_id, 3]), +-1 with probability
    1/2, layout [2 chains][n_T walkers][N sites] ("hot start").
  * inverse temperatures: geometric ladder beta_n = beta_min alpha^(n-1),
    alpha = (beta_max/beta_min)^(1/(N_T-1)) (Table I caption), ascending, so
    slot 0 is the hottest.  "T in [a, b]" gives beta_min = 1/b, beta_max = 1/a.
  * site index i = x + L (y + L z).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

J_GAUSS, J_PM1 = 0, 1
GRID = 2.0 ** -18
JMAX_UNITS = 2 ** 21 - 1


def geometric_betas(n_T: int, t_min: float, t_max: float) -> np.ndarray:
    return beta_ladder(n_T, 1.0 / t_max, 1.0 / t_min)


def beta_ladder(n_T: int, b_min: float, b_max: float) -> np.ndarray:
    """beta_n = beta_min alpha^n, alpha = (beta_max/beta_min)^(1/(n_T-1)),
    n = 0 .. n_T-1 (Table I caption)."""
    if n_T == 1:
        return np.array([b_min], dtype=np.float64)
    alpha = (b_max / b_min) ** (1.0 / (n_T - 1))
    return np.array([b_min * alpha ** n for n in range(n_T)], dtype=np.float64)


def gaussian_couplings(seed: int, sample_id: int, L: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, sample_id, 2])))
    g = rng.standard_normal(3 * L ** 3)
    n = np.clip(np.rint(g / GRID), -JMAX_UNITS, JMAX_UNITS)
    return (n * GRID).astype(np.float32).reshape(3, L ** 3)


def pm1_couplings(seed: int, sample_id: int, L: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, sample_id, 2])))
    b = rng.integers(0, 2, size=3 * L ** 3)
    return np.where(b == 0, 1, -1).astype(np.int8).reshape(3, L ** 3)


def initial_spins(seed: int, sample_id: int, L: int, n_T: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, sample_id, 3])))
    b = rng.integers(0, 2, size=2 * n_T * L ** 3)
    return np.where(b == 0, 1, -1).astype(np.int8).reshape(2, n_T, L ** 3)


@dataclass
class Workload:
    """A batch of disorder samples in the concatenated layout the C ABI takes."""
    L: np.ndarray                 # [S] int32
    n_temps: np.ndarray           # [S] int32
    h: np.ndarray                 # [S] float32
    sample_id: np.ndarray         # [S] uint32
    jkind: int
    seed: int
    measure_every: int
    measure_start: int
    beta: np.ndarray              # concat [S][n_T] float64
    J: np.ndarray                 # concat [S][3][N] float32 or int8
    spins0: np.ndarray            # concat [S][2][n_T][N] int8
    name: str = ""
    sweeps: int = 0
    beta_off: np.ndarray = field(default=None)
    J_off: np.ndarray = field(default=None)
    spin_off: np.ndarray = field(default=None)

    def __post_init__(self):
        N = self.L.astype(np.int64) ** 3
        self.beta_off = np.concatenate([[0], np.cumsum(self.n_temps.astype(np.int64))])
        self.J_off = np.concatenate([[0], np.cumsum(3 * N)])
        self.spin_off = np.concatenate([[0], np.cumsum(2 * self.n_temps.astype(np.int64) * N)])

    @property
    def n_samples(self) -> int:
        return int(len(self.L))

    def beta_of(self, s):
        return self.beta[self.beta_off[s]:self.beta_off[s + 1]]

    def J_of(self, s):
        N = int(self.L[s]) ** 3
        return self.J[self.J_off[s]:self.J_off[s + 1]].reshape(3, N)

    def spins0_of(self, s):
        N = int(self.L[s]) ** 3
        return self.spins0[self.spin_off[s]:self.spin_off[s + 1]].reshape(2, int(self.n_temps[s]), N)

    def attempts_per_sweep(self) -> int:
        return int((self.L.astype(np.int64) ** 3 * 2 * self.n_temps).sum())

    def subset(self, samples) -> "Workload":
        """The same samples (same ids, hence the same random streams)."""
        samples = list(samples)
        return Workload(
            L=self.L[samples].copy(), n_temps=self.n_temps[samples].copy(),
            h=self.h[samples].copy(), sample_id=self.sample_id[samples].copy(),
            jkind=self.jkind, seed=self.seed, measure_every=self.measure_every,
            measure_start=self.measure_start,
            beta=np.concatenate([self.beta_of(s) for s in samples]),
            J=np.concatenate([self.J_of(s).ravel() for s in samples]),
            spins0=np.concatenate([self.spins0_of(s).ravel() for s in samples]),
            name=self.name + "[subset]", sweeps=self.sweeps)


def make_workload(Ls, n_temps, t_range, hs, jkind=J_GAUSS, seed=1, sample_ids=None,
                  measure_every=10, measure_start=0, name="", sweeps=0, beta_range=None) -> Workload:
    """Per-sample lists (or scalars broadcast to S = len(Ls)).  The ladder is
    geometric in beta over T in t_range, or over beta in beta_range if given."""
    S = len(Ls)
    n_temps = np.broadcast_to(np.asarray(n_temps, dtype=np.int32), (S,)).copy()
    hs = np.broadcast_to(np.asarray(hs, dtype=np.float32), (S,)).copy()
    Ls = np.asarray(Ls, dtype=np.int32)
    ids = np.arange(S, dtype=np.uint32) if sample_ids is None else np.asarray(sample_ids, dtype=np.uint32)
    betas, Js, sp = [], [], []
    for s in range(S):
        L, nT, sid = int(Ls[s]), int(n_temps[s]), int(ids[s])
        betas.append(beta_ladder(nT, *beta_range) if beta_range is not None else geometric_betas(nT, *t_range))
        if jkind == J_GAUSS:
            Js.append(gaussian_couplings(seed, sid, L).ravel())
        else:
            Js.append(pm1_couplings(seed, sid, L).ravel())
        sp.append(initial_spins(seed, sid, L, nT).ravel())
    return Workload(L=Ls, n_temps=n_temps, h=hs, sample_id=ids, jkind=jkind, seed=seed,
                    measure_every=measure_every, measure_start=measure_start,
                    beta=np.concatenate(betas), J=np.concatenate(Js),
                    spins0=np.concatenate(sp), name=name, sweeps=sweeps)


# The five workloads (lattice sizes, ladders, fields and sample counts of the
# paper's production shapes, scaled to one GPU).  ``samples`` may shrink a
# workload for tests; sample ids stay those of the full workload.
CONFIGS = {
    "L4_gauss": dict(L=4, S=16, n_T=8, T=(0.5, 2.0), h=0.3, jkind=J_GAUSS, sweeps=5000),
    "L8_gauss": dict(L=8, S=1024, n_T=16, T=(0.6, 1.6), h=0.2, jkind=J_GAUSS, sweeps=10000),
    "mixed_L6_12": dict(L=None, S=4096, n_T=16, T=(0.5, 1.6), h=None, jkind=J_GAUSS, sweeps=10000),
    "L16_gauss": dict(L=16, S=2048, n_T=24, T=(0.4, 1.5), h=0.1, jkind=J_GAUSS, sweeps=20000),
    "L32_pm1": dict(L=32, S=512, n_T=32, T=(0.5, 2.0), h=0.4, jkind=J_PM1, sweeps=5000),
}


def config_workload(name: str, samples=None, seed: int = 1, measure_every: int = 10,
                    measure_start=None) -> Workload:
    c = CONFIGS[name]
    S = c["S"]
    ids = list(range(S)) if samples is None else list(samples)
    if name == "mixed_L6_12":
        Ls = [[6, 8, 10, 12][j % 4] for j in ids]
        hs = [[0.1, 0.2, 0.3][(j // 4) % 3] for j in ids]
    else:
        Ls = [c["L"]] * len(ids)
        hs = [c["h"]] * len(ids)
    ms = c["sweeps"] // 2 if measure_start is None else measure_start
    return make_workload(Ls, c["n_T"], c["T"], hs, jkind=c["jkind"], seed=seed,
                         sample_ids=ids, measure_every=measure_every, measure_start=ms,
                         name=name, sweeps=c["sweeps"])
