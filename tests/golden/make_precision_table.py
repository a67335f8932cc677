"""Write tests/golden/precision_mirror_vs_fp64.json: the precision statement.

The engine computes local fields and the Metropolis test in binary32 (the
oracle's "mirror" mode, which the GPU path matches bit for bit) and keeps
energies exact and accumulators in binary64.  The oracle's binary64 mode runs
the same Markov chain with binary64 fields, libm exp and 53-bit uniforms (its
own random stream).  From the same initial states the two give the same
expected value of every time-averaged observable, so their difference on the
same disorder samples, divided by its paired leave-one-sample-out jackknife
error, is a z-score that stays of order one unless binary32 biases a result.

This script calls only the oracle.  For each workload shape (the L = 8 and the
L = 16 Gaussian workloads, 32 samples each, 2000 sweeps, measurements every
10 sweeps over the second half) it records, per observable of eqs. 3-6 and per
temperature slot: the mirror value, the binary64 value, their difference, the
paired jackknife error and z.

    python tests/golden/make_precision_table.py [--threads 8]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ea_oracle as O  # noqa: E402
from paper_1403_4560_amd import workload as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_mirror_vs_fp64.json")
KEYS = ("q", "chi0", "chi_kmin", "chi_k2", "g", "xi_L", "R12", "chi0_over_chikmin", "E_a", "E_b")
CASES = [dict(config="L8_gauss", samples=32, sweeps=2000, measure_every=10),
         dict(config="L16_gauss", samples=32, sweeps=2000, measure_every=10)]


def paired_jackknife(acc_a, acc_b, L):
    """Per observable: (difference of the two runs' observables over the same
    samples, its leave-one-sample-out jackknife error)."""
    S = acc_a.shape[0]
    fa, fb = O.observables(acc_a, L), O.observables(acc_b, L)
    reps = [(O.observables(np.delete(acc_a, s, axis=0), L), O.observables(np.delete(acc_b, s, axis=0), L))
            for s in range(S)]
    out = {}
    for k in KEYS:
        diff = fa[k] - fb[k]
        R = np.stack([ra[k] - rb[k] for ra, rb in reps])
        err = np.sqrt((S - 1) / S * ((R - R.mean(axis=0)) ** 2).sum(axis=0))
        out[k] = (fa[k], fb[k], diff, err)
    return out


def run_case(c, threads):
    work = W.config_workload(c["config"], samples=range(c["samples"]), measure_every=c["measure_every"],
                             measure_start=c["sweeps"] // 2)
    L = int(work.L[0])
    acc = {}
    for mode in (O.MODE_MIRROR, O.MODE_FP64):
        t0 = time.time()
        ens = O.OracleEnsemble(work, mode=mode).run(c["sweeps"], threads=threads)
        acc[mode] = np.stack([st.acc for st in ens.states])
        print("%s mode %d: %.1f s" % (c["config"], mode, time.time() - t0), flush=True)
    res = paired_jackknife(acc[O.MODE_MIRROR], acc[O.MODE_FP64], L)
    obs = {}
    zs = []
    with np.errstate(invalid="ignore", divide="ignore"):
        for k, (a, b, d, e) in res.items():
            z = np.where((e > 0) & np.isfinite(d), d / e, np.nan)
            zs.extend(np.abs(z[np.isfinite(z)]).tolist())
            obs[k] = {"mirror": a.tolist(), "binary64": b.tolist(), "diff": d.tolist(), "err": e.tolist(),
                      "z": z.tolist()}
    zs = np.array(zs)
    summary = {"comparisons": int(zs.size), "max_abs_z": float(zs.max()),
               "rms_z": float(np.sqrt((zs ** 2).mean()))}
    print(c["config"], summary, flush=True)
    return {"case": c, "L": L, "n_T": int(work.n_temps[0]), "h": float(work.h[0]),
            "beta": [float(x) for x in work.beta_of(0)], "summary": summary, "observables": obs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    table = {"what": "mirror (binary32 fields and acceptance) minus binary64 mode, same samples and initial "
                     "states, paired leave-one-sample-out jackknife z per observable and slot",
             "cases": [run_case(c, args.threads) for c in CASES]}
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
