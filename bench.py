"""Benchmark: Metropolis + parallel-tempering throughput on one MI355X.

Workload (the L = 16 LDS-resident shape): 2048 Gaussian-coupling samples
(couplings on the 2^-18 grid), L = 16, 24 temperatures geometric in
T = [0.4, 1.5], two replicas per temperature, h = 0.1, overlap measurement
every 10 sweeps (measuring from the first sweep, so the timed region is the
production measuring phase).  Inputs are seeded synthetic arrays, resident in
HBM before timing starts.

One step = one chunk of 100 sweeps of the whole batch: 2 x 100 checkerboard
half-sweeps of every walker, 100 replica-exchange passes, 10 overlap
measurements of every slot.  The metric is spin-flip attempts per ns
(one attempt = one Metropolis trial at one site of one walker).

Prints one JSON line (rank 0).  Besides the headline value it reports the
unbatched form (the same kernels, one launch per sample, on a 64-sample subset,
and, for L divisible by 8, the HBM-resident kernels that spread one sample's
walkers over many workgroups, one sample per launch, on 16 samples),
the roofline of the dominant kernel from HIP events recorded around each of
its launches, and the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/ns at L=16 batched vs unbatched; bit-exact spins"
SWEEPS_PER_STEP = 100
KERNEL = {"L16_gauss": "row_sweep_kernel<16, 0>", "L8_gauss": "row_sweep_kernel<8, 0>",
          "L4_gauss": "site_sweep_kernel<4, 0, 0>", "mixed_L6_12": "group/row sweep kernels (4 sizes)",
          "L32_pm1": "bits_sweep_kernel<32, 0>"}
WORKLOAD_TEXT = {
    "L16_gauss": "L16_gauss: L=16, 2048 samples, 24 temperatures geometric in T=[0.4,1.5], 2 replicas, "
                 "Gaussian J on the 2^-18 grid, h=0.1, measure every 10 sweeps",
    "L4_gauss": "L4_gauss: L=4, 16 samples, 8 temperatures in T=[0.5,2.0], 2 replicas, Gaussian J, h=0.3",
    "L8_gauss": "L8_gauss: L=8, 1024 samples, 16 temperatures in T=[0.6,1.6], 2 replicas, Gaussian J, h=0.2",
    "mixed_L6_12": "mixed_L6_12: 4096 samples, L in {6,8,10,12}, h in {0.1,0.2,0.3}, 16 temperatures in "
                   "T=[0.5,1.6], 2 replicas, Gaussian J",
    "L32_pm1": "L32_pm1: L=32, 512 samples, 32 temperatures in T=[0.5,2.0], 2 replicas, +-1 J, h=0.4, "
               "one bit per spin in LDS",
}

# Algorithmic work of one Metropolis attempt: the VALU instructions (one lane
# each) that a minimal gfx950 implementation of the numeric contract issues,
# per 4-site word (one Philox call), divided by 4.
#   Philox4x32-10: 10 rounds x (2 32x32->64 multiply-adds + 2 three-input
#     xors), less the 3 that depend only on (walker, sweep): the counter's
#     word 2 product and xor of round 0 and the word 0 product of round 1 = 37
#   shifted x-neighbour word (one byte permute)                        =  1
#   per site, Gaussian couplings: 6 byte-select multiplies and 3 adds for
#     S_u plus the field's grid part, conversion (1), one fused operation for
#     the temperature and the field remainder (1), the spin's sign (1),
#     hardware exponential (1), word to float (1), the acceptance gap (1)
#                                                              = 15 x 4 = 60
#   the word's spin-sign mask (1)                                      =  1
#   flip mask from the gaps' sign bits: 2 byte permutes and 1 and       =  3
#   exact-path test: least |gap| by 2 three-way minimums, 1 compare     =  3
#   word tail: new spins (1), flip and down-flip counts (3)            =  4
#   energy, second half-sweep only: per site sign-extend and xor (2), two
#     adds per word, down count (2): 12 per word, 6 on average        =  6
# Gaussian: (37 + 1 + 60 + 1 + 3 + 3 + 4 + 6) / 4 = 28.75.
# +-1 couplings, one bit per spin, per 32-site word / 32:
#   Philox 8 x 37 = 296; per site: table address (1), compare and carry-in
#   (2) = 96; class bytes: 3 spread-table addresses (2 each) and 4 merges per
#   8 sites = 40; neighbours (x rotations 6, x selects 2, y funnels 2), six
#   unsatisfied-bond words (6), the count c (8), dE <= 0 (8), class planes
#   (3), new spins (1), flip and down-flip counts (3), energy on the second
#   half only (7, 3.5 on average) = 42.5: 474.5 / 32 = 14.83.
BYTE_PM1_OPS_PER_ATTEMPT = 25.5
ALG_OPS_PER_ATTEMPT = {"L16_gauss": 28.75, "L8_gauss": 28.75, "mixed_L6_12": 28.75, "L4_gauss": 28.75,
                       "L32_pm1": 474.5 / 32}
# Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = non-packed VALU lane-instructions/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# HBM bytes of one launch of the dominant kernel from hardware counters
# (FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0, the factors a plain copy of
# known size reads), keyed by a fingerprint of the kernel sources they were
# taken on; reported as null once the kernels change.
MEASURED_TRAFFIC = {"L16_gauss": ("b11a8e83f689c066", 2.2589e9), "L32_pm1": ("b11a8e83f689c066", 3.5384e9)}
KERNEL_SOURCES = tuple("paper_1403_4560_amd/csrc/" + f for f in (
    "ea_kernels.hip", "ea_bits.hip", "ea_group.hip", "ea_item.hpp", "ea_update.hpp", "ea_device.hpp",
    "ea_types.hpp"))


def kernel_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def cpu_baseline(work, n_samples, attempts):
    from oracle import ea_oracle as O
    threads = min(16, os.cpu_count() or 1)
    sub = work.subset(range(min(n_samples, work.n_samples)))
    n_samples = sub.n_samples
    sweeps = max(1, int(round(attempts / sub.attempts_per_sweep())))
    ens = O.OracleEnsemble(sub)
    t0 = time.perf_counter()
    ens.run(sweeps, threads=threads)
    dt = time.perf_counter() - t0
    attempts = sub.attempts_per_sweep() * sweeps
    return {"value": attempts / dt / 1e9, "unit": "attempts/ns", "cores": threads, "kind": "oracle",
            "sample": "%d of the %d samples x %d sweeps (%.3g attempts), %.1f s wall on %d threads"
                      % (n_samples, work.n_samples, sweeps, attempts, dt, threads)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="L16_gauss",
                    help="L16_gauss (default), L4_gauss, L8_gauss, mixed_L6_12 or L32_pm1")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--unbatched-samples", type=int, default=64)
    ap.add_argument("--unbatched-steps", type=int, default=2)
    ap.add_argument("--cpu-samples", type=int, default=64)
    ap.add_argument("--cpu-attempts", type=float, default=7.5e8,
                    help="size of the CPU oracle sample (about 10-30 s of single-core work per 1e8)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-unbatched", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time candidate plans first (the L=16 row engine has no thread-count knob)")
    ap.add_argument("--tier", type=int, default=0,
                    help="0 automatic (default); 1 HBM-resident for L divisible by 8; 2 no one-bit engine; "
                         "3 one-site-per-thread engine (comparisons only)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="before timing, run a plain device-to-device copy of this many bytes "
                         "(a reference kernel of known traffic for hardware byte counters)")
    ap.add_argument("--peaks", action="store_true",
                    help="print the measured rates of the roofline's units (VALU issue of xor, 64-bit "
                         "multiply-add and high multiply; LDS read and HBM copy bandwidth) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every disorder sample is independent, so more GPUs "
              "would each run their own share of samples; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1403_4560_amd import binding, workload as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.peaks:
        r = binding.measure_peaks()
        print(json.dumps({"peaks_measured": {
            "valu_xor_Tops": r["valu_xor_ops"] / 1e12, "valu_mad_u64_Tops": r["valu_mad_u64_ops"] / 1e12,
            "valu_mul_hi_Tops": r["valu_mul_hi_ops"] / 1e12, "lds_read_TBps": r["lds_read_bytes"] / 1e12,
            "hbm_copy_TBps": r["hbm_copy_bytes"] / 1e12, "valu_exp_Tops": r["valu_exp_ops"] / 1e12},
            "derived_valu_peak_Tops": VALU_PEAK_TOPS, "published_hbm_TBps": 8.0}))
        return
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    work = W.config_workload(args.workload, measure_start=0, measure_every=10)
    ens = binding.Ensemble(work, stream=stream.cuda_stream, tier=args.tier)
    ens.set_plan(chunk=SWEEPS_PER_STEP)
    plan = ens.autotune(trial_sweeps=4) if args.autotune else ens.get_plan()
    ens.set_plan(chunk=SWEEPS_PER_STEP)
    attempts_per_step = work.attempts_per_sweep() * SWEEPS_PER_STEP
    progress("ensemble ready, plan threads=%d" % plan.threads)

    for _ in range(args.warmup):
        ens.sweep_pt(SWEEPS_PER_STEP)
    ens.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ens.sweep_pt(SWEEPS_PER_STEP)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_launches = ens.kernel_time()
    ens.set_timing(False)
    assert ens.check_energies() == 0, "incremental energies diverged"
    value = attempts_per_step * args.steps / (dt * 1e9)
    ens.close()
    progress("timed %d steps in %.2f s: %.1f attempts/ns" % (args.steps, dt, value))

    # roofline of the dominant kernel (the LDS-resident sweep kernel of the workload)
    avg_launch_s = k_ms / 1e3 / max(k_launches, 1)
    attempts_per_launch = attempts_per_step  # one launch per step (chunk)
    ops = ALG_OPS_PER_ATTEMPT[args.workload]
    if work.jkind == 1 and args.tier != 0:
        ops = BYTE_PM1_OPS_PER_ATTEMPT  # +-1 couplings on the byte engines
    fp, traffic = MEASURED_TRAFFIC.get(args.workload, (None, None)) if args.tier == 0 else (None, None)
    if fp != kernel_fingerprint():
        traffic = None
    kernel = KERNEL.get(args.workload, "sweep kernels") if args.tier == 0 else "tier %d kernels" % args.tier
    achieved = attempts_per_launch * ops / avg_launch_s / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                "kernel": kernel, "avg_launch_ms": avg_launch_s * 1e3,
                "ops_per_attempt": ops, "traffic_unit": "HBM bytes per launch (hardware counters)"}

    unbatched = None
    if not args.no_unbatched:
        sub = work.subset(range(min(args.unbatched_samples, work.n_samples)))
        ub = binding.Ensemble(sub, stream=stream.cuda_stream, tier=args.tier)
        ub.set_plan(chunk=SWEEPS_PER_STEP, threads=plan.threads)
        ub.sweep_pt_unbatched(SWEEPS_PER_STEP)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.unbatched_steps):
            ub.sweep_pt_unbatched(SWEEPS_PER_STEP)
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        ub.close()
        ub_value = sub.attempts_per_sweep() * SWEEPS_PER_STEP * args.unbatched_steps / (dt1 * 1e9)
        progress("unbatched: %.1f attempts/ns" % ub_value)
        unbatched = {"value": ub_value, "unit": "attempts/ns", "samples": sub.n_samples,
                     "sweeps": SWEEPS_PER_STEP * args.unbatched_steps,
                     "batched_over_unbatched": value / ub_value}
        if all(int(L) % 8 == 0 for L in work.L):
            # the stronger one-sample-per-launch form: the HBM-resident kernels
            # spread one sample's walkers over many workgroups per launch
            sub2 = work.subset(range(min(16, work.n_samples)))
            ub2 = binding.Ensemble(sub2, stream=stream.cuda_stream, tier=1)
            ub2.sweep_pt_unbatched(10)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ub2.sweep_pt_unbatched(SWEEPS_PER_STEP)
            torch.cuda.synchronize()
            dt2 = time.perf_counter() - t2
            ub2.close()
            v2 = sub2.attempts_per_sweep() * SWEEPS_PER_STEP / (dt2 * 1e9)
            progress("unbatched, HBM-resident spread: %.1f attempts/ns" % v2)
            unbatched["spread_form"] = {"value": v2, "samples": sub2.n_samples, "sweeps": SWEEPS_PER_STEP,
                                        "batched_over_spread": value / v2,
                                        "kernels": "HBM-resident half-sweep, exchange, snapshot per sweep"}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(work, args.cpu_samples, args.cpu_attempts)
        progress("cpu oracle: %.4f attempts/ns" % cpu["value"])

    line = {
        "metric": METRIC, "value": value, "unit": "attempts/ns", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "sweeps_per_step": SWEEPS_PER_STEP, "samples": work.n_samples,
                   "attempts_per_step": attempts_per_step, "threads_per_workgroup": plan.threads,
                   "tier": args.tier,
                   "parallelism": "samples x chains across workgroups"},
        "unbatched": unbatched,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
