"""Production driver in the shape of the paper's simulations (Table I).

Table I runs +-1 couplings at L = 6, 8, 10 with N_T = 56 temperatures
geometric in beta over [0.1, 1.8], in a field h = 0.1, two replicas per
temperature, 2e6 sweeps per replica, the first half for thermalization and
the second half for measurement; the paper checks equilibration with the
logarithmic binning test (caption of the figure of R12 against the number of
sweeps at L = 10, beta = 1.8).  This driver runs that shape, with the sample
count and run length the caller chooses, on the device engine.

Measurements are binned logarithmically in time: bin k holds the
measurements taken in sweeps (2^k, 2^(k+1)].  The accumulators (and the flip
and exchange counters) are reset when a bin starts, so each bin's disorder
averages and jackknife errors come from that bin alone; the last bin is the
second half of the run, the paper's measuring window.  A run passes the test
when the last three bins agree within their errors.

    python -m paper_1403_4560_amd.driver --L 10 --samples 256 --log2-sweeps 14 --out run.json
"""
import argparse
import json
import math
import sys
from dataclasses import dataclass, field

import numpy as np

from . import binding
from . import workload as W

TABLE_I = {  # L: disorder samples and sweeps per replica in the paper's runs
    6: dict(samples=500_000, sweeps=2_000_000),
    8: dict(samples=350_000, sweeps=2_000_000),
    10: dict(samples=240_000, sweeps=2_000_000),
}
TABLE_I_NT = 56
TABLE_I_BETA = (0.1, 1.8)
FIELD = 0.1


def table1_workload(L: int, samples: int, seed: int = 1, first_sample: int = 0, h: float = FIELD,
                    n_T: int = TABLE_I_NT, beta_range=TABLE_I_BETA, measure_every: int = 10) -> W.Workload:
    """+-1 couplings, the Table I ladder and field, `samples` disorder
    realizations with logical ids first_sample, first_sample + 1, ..."""
    ids = list(range(first_sample, first_sample + samples))
    return W.make_workload([L] * samples, n_T, None, h, jkind=W.J_PM1, seed=seed, sample_ids=ids,
                           measure_every=measure_every, measure_start=0, beta_range=beta_range,
                           name="table1-L%d" % L)


@dataclass
class Bin:
    k: int
    first_sweep: int                   # bin covers sweeps (first_sweep, last_sweep]
    last_sweep: int
    measurements: int                  # per slot
    obs: dict = field(default_factory=dict)     # name -> (value[n_T], error[n_T])
    swap_rate: np.ndarray = None       # accepted exchanges per attempt, per pair (t, t+1)
    flip_rate: np.ndarray = None       # accepted flips per attempt, per slot

    def to_json(self):
        return {"k": self.k, "sweeps": [self.first_sweep, self.last_sweep], "measurements": self.measurements,
                "obs": {n: {"value": v.tolist(), "error": e.tolist()} for n, (v, e) in self.obs.items()},
                "swap_rate": self.swap_rate.tolist(), "flip_rate": self.flip_rate.tolist()}


def exchange_attempts(lo: int, hi: int, t: int) -> int:
    """Sweeps n in [lo, hi) after which pair (t, t+1) is offered an exchange
    (n = t mod 2)."""
    r = t & 1
    return (hi - r + 1) // 2 - (lo - r + 1) // 2


def first_bin_for(measure_every: int) -> int:
    """Smallest k whose bin (2^k, 2^(k+1)] holds at least two measurements."""
    k = 0
    while (2 ** (k + 1)) // measure_every - (2 ** k) // measure_every < 2:
        k += 1
    return k


def run_log_binned(work: W.Workload, log2_sweeps: int, first_bin: int | None = None, stream=None,
                   progress=None) -> list:
    """Run 2^log2_sweeps sweeps of every sample of `work` (one lattice size and
    ladder length) and return the bins k = first_bin .. log2_sweeps - 1."""
    Ls, nTs = set(int(x) for x in work.L), set(int(x) for x in work.n_temps)
    if len(Ls) != 1 or len(nTs) != 1:
        raise ValueError("one lattice size and one ladder length per run")
    L, n_T = Ls.pop(), nTs.pop()
    if work.n_samples < 2:
        raise ValueError("the jackknife needs at least two samples")
    m = work.measure_every
    if m < 1:
        raise ValueError("measurements are required (measure_every >= 1)")
    k0 = first_bin_for(m) if first_bin is None else first_bin
    if k0 >= log2_sweeps:
        raise ValueError("log2_sweeps must exceed the first bin %d" % k0)
    N = L ** 3
    bins = []
    with binding.Ensemble(work, stream=stream) as ens:
        ens.sweep_pt(2 ** k0)  # sweeps (0, 2^k0]: thermalization only
        for k in range(k0, log2_sweeps):
            lo, hi = 2 ** k, 2 ** (k + 1)
            ens.reset_accumulators()
            ens.sweep_pt(hi - lo)
            ms = ens.measure()
            nmeas = hi // m - lo // m
            acc0 = np.stack([a[:, 0] for a in ms["acc"]])
            if not np.all(acc0 == nmeas):
                raise RuntimeError("bin %d: expected %d measurements per slot" % (k, nmeas))
            obs = ens.finalize_jackknife()
            swaps = np.stack(ms["swaps"]).astype(np.float64)     # [S][2][n_T]
            flips = np.stack(ms["flips"]).astype(np.float64)
            attempts = np.array([exchange_attempts(lo, hi, t) for t in range(n_T)], dtype=np.float64)
            with np.errstate(invalid="ignore", divide="ignore"):
                swap_rate = swaps.sum(axis=(0, 1))[:-1] / (2 * work.n_samples * attempts[:-1])
            flip_rate = flips.sum(axis=(0, 1)) / (2.0 * work.n_samples * (hi - lo) * N)
            bins.append(Bin(k, lo, hi, nmeas, obs, swap_rate, flip_rate))
            if progress:
                progress(bins[-1])
    return bins


def bins_agree(bins: list, name: str = "R12", slot: int = -1, last: int = 3, nsigma: float = 1.0) -> bool:
    """Logarithmic binning test: the last `last` bins agree pairwise within
    nsigma combined standard errors for observable `name` at `slot`."""
    if len(bins) < last:
        return False
    tail = bins[-last:]
    vals = [(b.obs[name][0][slot], b.obs[name][1][slot]) for b in tail]
    for i in range(last):
        for j in range(i + 1, last):
            (a, ea), (b, eb) = vals[i], vals[j]
            if not (math.isfinite(a) and math.isfinite(b)):
                return False
            if abs(a - b) > nsigma * math.sqrt(ea * ea + eb * eb):
                return False
    return True


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", type=int, choices=sorted(TABLE_I), required=True)
    ap.add_argument("--samples", type=int, default=64)
    ap.add_argument("--first-sample", type=int, default=0)
    ap.add_argument("--log2-sweeps", type=int, default=12)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--measure-every", type=int, default=10)
    ap.add_argument("--observable", default="R12")
    ap.add_argument("--out", default=None, help="write the bins as JSON")
    args = ap.parse_args(argv)
    import torch  # device memory and streams
    torch.cuda.set_device(0)
    work = table1_workload(args.L, args.samples, seed=args.seed, first_sample=args.first_sample,
                           measure_every=args.measure_every)

    def show(b):
        v, e = b.obs[args.observable]
        print("bin %2d sweeps (%d, %d]: %s(beta=%.3f) = %.5g +- %.2g" %
              (b.k, b.first_sweep, b.last_sweep, args.observable, work.beta_of(0)[-1], v[-1], e[-1]),
              file=sys.stderr, flush=True)

    bins = run_log_binned(work, args.log2_sweeps, stream=torch.cuda.current_stream().cuda_stream, progress=show)
    ok = bins_agree(bins, args.observable)
    print("logarithmic binning test (%s, last three bins, 1 sigma): %s" %
          (args.observable, "passed" if ok else "not passed"), file=sys.stderr)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"L": args.L, "samples": args.samples, "n_T": TABLE_I_NT, "beta": work.beta_of(0).tolist(),
                       "h": FIELD, "seed": args.seed, "log2_sweeps": args.log2_sweeps,
                       "passed": ok, "bins": [b.to_json() for b in bins]}, f)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
