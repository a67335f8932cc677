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

The timed region replays each chunk from its captured hipGraph (the production
path); an untimed pass of direct launches then records HIP events around the
sweep kernels of every chunk for the roofline.

Prints one JSON line (rank 0).  Besides the headline value it reports the
unbatched form (the same kernels, one launch per sample, on a 64-sample subset,
and, for L divisible by 8, the HBM-resident kernels that spread one sample's
walkers over many workgroups, one sample per launch, on 16 samples), the
roofline of the dominant kernel (against the derived VALU peak and against the
unit rates measured in-process, with its LDS traffic), the CPU oracle on a
bounded sample (with the host's CPU model), and the same figures for the
other workload shapes (L8_gauss, mixed_L6_12, L32_pm1) under other_workloads.
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
MEASURED_TRAFFIC = {"L16_gauss": ("bbc1b9be80475284", 2.0324e9), "L32_pm1": ("bbc1b9be80475284", 3.5397e9),
                    "mixed_L6_12": ("bbc1b9be80475284", 0.7665e9), "L8_gauss": ("bbc1b9be80475284", 0.1367e9)}
KERNEL_SOURCES = tuple("paper_1403_4560_amd/csrc/" + f for f in (
    "ea_kernels.hip", "ea_bits.hip", "ea_group.hip", "ea_batch.hip", "ea_row.hpp", "ea_group.hpp", "ea_item.hpp",
    "ea_update.hpp", "ea_device.hpp", "ea_types.hpp"))


def kernel_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# Instruction mix of the algorithmic count per attempt, priced at the unit
# rates measured on the device (ea_measure_peaks): 32x32->64 multiply-adds,
# hardware exponentials and simple 32-bit operations.
#   Gaussian, per 4-site word: Philox 18 multiply-adds; 4 exponentials; the
#     other 93 operations simple (115 in all).
#   +-1 one bit per spin, per 32-site word: 8 Philox calls = 144 multiply-adds,
#     330.5 simple (474.5 in all).
OP_MIX = {"gauss": {"mad": 18 / 4, "exp": 4 / 4, "simple": 93 / 4},
          "bits": {"mad": 144 / 32, "exp": 0.0, "simple": 330.5 / 32}}
# LDS bytes one attempt reads and writes by design (the dominant kernel):
#   row engine, per 4-site word: 7 spin words (28 B), 6 coupling vectors of 4
#     int32 (96 B) and on half the words one more coupling (2 B on average),
#     the updated word (4 B): 130 B / 4;
#   group engine, per site of a quad (4 attempts): own and 6 neighbour words
#     (28 B), the neighbour table entry (16 B), 6 couplings (24 B), the store
#     (4 B): 72 B / 4;
#   one-bit engine, per 32-site word: own, 4 neighbour words and the x word
#     (24 B), 6 bond words (24 B), 8 threshold reads per 8 sites, 3 spreading
#     reads per 8 sites (44 B), the store (4 B): 96 B / 32.
LDS_BYTES_PER_ATTEMPT = {"row": 130 / 4, "group": 72 / 4, "bits": 96 / 32}
# LDS read bandwidth: 256 B per clock per CU on gfx950 (twice CDNA3's 128 B; the
# measured 16-byte read rate, about 245 B per clock per CU, agrees)
LDS_PEAK_TBPS = 256 * 256 * 2.4e9 / 1e12
HBM_PEAK_TBPS = 8.0
EXTRA_WORKLOADS = ("L8_gauss", "mixed_L6_12", "L32_pm1")
ENGINE_OF = {"L16_gauss": "row", "L8_gauss": "row", "mixed_L6_12": "group", "L4_gauss": "group",
             "L32_pm1": "bits"}


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


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
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "%d of the %d samples x %d sweeps (%.3g attempts), %.1f s wall on %d threads"
                      % (n_samples, work.n_samples, sweeps, attempts, dt, threads)}


def measured_peak_tops(mix, peaks):
    """Lane-operations per second the kernel's instruction mix allows at the
    measured unit rates (a harmonic mean weighted by the mix)."""
    n = mix["mad"] + mix["exp"] + mix["simple"]
    t = (mix["mad"] / peaks["valu_mad_u64_ops"] + mix["exp"] / peaks["valu_exp_ops"] +
         mix["simple"] / peaks["valu_xor_ops"])
    return n / t / 1e12


def time_workload(binding, work, stream, steps, warmup, tier=0, timing_steps=3, autotune=True, batch=None):
    """Graph-replayed steps timed by the host clock (the production path), then
    an untimed pass of direct launches with HIP events around the sweep
    kernels of every chunk, for the roofline.  The plan is autotuned first
    (outside the timed region); batch=False then runs every lattice-size class
    in a launch of its own (per-class kernel counters)."""
    import torch
    ens = binding.Ensemble(work, stream=stream.cuda_stream, tier=tier)
    plan = ens.autotune(trial_sweeps=4) if autotune else ens.get_plan()
    ens.set_plan(chunk=SWEEPS_PER_STEP, use_graph=True, batch=batch)
    plan = ens.get_plan()
    bplan = ens.batch_plan()
    for _ in range(warmup):
        ens.sweep_pt(SWEEPS_PER_STEP)  # the first call captures the chunk's graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ens.sweep_pt(SWEEPS_PER_STEP)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ens.set_timing(True)
    t1 = time.perf_counter()
    for _ in range(timing_steps):
        ens.sweep_pt(SWEEPS_PER_STEP)
    torch.cuda.synchronize()
    dt_direct = time.perf_counter() - t1
    k_ms, k_launches = ens.kernel_time()
    ens.set_timing(False)
    bad = ens.check_energies()
    engines = sorted(set(ens.engines()))
    ens.close()
    assert bad == 0, "incremental energies diverged"
    # the events bracket the sweep kernels of each chunk: one launch, or with
    # class launches all of them (their summed time per chunk)
    return {"dt": dt, "ms_per_step": dt * 1e3 / steps, "direct_ms_per_step": dt_direct * 1e3 / timing_steps,
            "avg_launch_s": k_ms / 1e3 / max(k_launches, 1), "engines": engines,
            "plan": {"batch_launch": bool(plan.batch), "site_threads": plan.threads,
                     "classes": [{"L": L, "engine": e, "items_per_workgroup": t}
                                 for L, e, t in zip(bplan["L"], bplan["engine"], bplan["teams"])]}}


def time_unbatched(binding, work, stream, n_samples, steps, tier=0):
    import torch
    sub = work.subset(range(min(n_samples, work.n_samples)))
    ub = binding.Ensemble(sub, stream=stream.cuda_stream, tier=tier)
    ub.set_plan(chunk=SWEEPS_PER_STEP)
    ub.sweep_pt_unbatched(SWEEPS_PER_STEP)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        ub.sweep_pt_unbatched(SWEEPS_PER_STEP)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t1
    ub.close()
    return {"value": sub.attempts_per_sweep() * SWEEPS_PER_STEP * steps / (dt1 * 1e9), "unit": "attempts/ns",
            "samples": sub.n_samples, "sweeps": SWEEPS_PER_STEP * steps}


def roofline_of(name, work, timed, tier, peaks):
    attempts_per_launch = work.attempts_per_sweep() * SWEEPS_PER_STEP  # one chunk per step
    avg = timed["avg_launch_s"]
    ops = ALG_OPS_PER_ATTEMPT[name]
    if work.jkind == 1 and tier != 0:
        ops = BYTE_PM1_OPS_PER_ATTEMPT  # +-1 couplings on the byte engines
    fp, traffic = MEASURED_TRAFFIC.get(name, (None, None)) if tier == 0 else (None, None)
    if fp != kernel_fingerprint():
        traffic = None
    kernel = KERNEL.get(name, "sweep kernels") if tier == 0 else "tier %d kernels" % tier
    achieved = attempts_per_launch * ops / avg / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
         "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
         "kernel": kernel, "avg_launch_ms": avg * 1e3,
         "ops_per_attempt": ops, "traffic_unit": "HBM bytes per launch (hardware counters)"}
    engine = ENGINE_OF.get(name, "group")
    if tier == 0 and peaks is not None:
        mp = measured_peak_tops(OP_MIX["bits" if engine == "bits" else "gauss"], peaks)
        r["frac_measured_peaks"] = achieved / mp
        r["measured_peak"] = mp
    if tier == 0:
        lb = LDS_BYTES_PER_ATTEMPT[engine]
        lds = attempts_per_launch * lb / avg / 1e12
        r["lds"] = {"bytes_per_attempt": lb, "achieved_TBps": lds, "peak_TBps": LDS_PEAK_TBPS,
                    "frac": lds / LDS_PEAK_TBPS}
        if peaks is not None:
            r["lds"]["frac_measured_peak"] = lds / (peaks["lds_read_bytes"] / 1e12)
    if traffic is not None:
        hbm = traffic / avg / 1e12
        r["hbm"] = {"achieved_TBps": hbm, "peak_TBps": HBM_PEAK_TBPS, "frac": hbm / HBM_PEAK_TBPS}
    return r


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
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (L8_gauss, mixed_L6_12, L32_pm1) after the headline")
    ap.add_argument("--extra-steps", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the plan autotuning done before each timed workload")
    ap.add_argument("--class-launches", action="store_true",
                    help="after autotuning, run each lattice-size class in a launch of its own (per-class "
                         "kernel counters of an uneven batch)")
    ap.add_argument("--tier", type=int, default=0,
                    help="0 automatic (default); 1 HBM-resident for L divisible by 8; 2 no one-bit engine; "
                         "3 one-site-per-thread engine (comparisons only)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="before timing, run a plain device-to-device copy of this many bytes "
                         "(a reference kernel of known traffic for hardware byte counters)")
    ap.add_argument("--peaks", action="store_true",
                    help="print the measured rates of the roofline's units (VALU issue of xor, 64-bit "
                         "multiply-add and high multiply; LDS read and HBM copy bandwidth) and exit")
    ap.add_argument("--no-peaks", action="store_true", help="skip the in-process unit-rate measurement")
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
    peaks = None
    if args.peaks or not args.no_peaks:
        peaks = binding.measure_peaks()
        progress("measured unit rates: xor %.1f T, mad %.1f T, exp %.1f T lane-ops/s, LDS %.0f TB/s"
                 % (peaks["valu_xor_ops"] / 1e12, peaks["valu_mad_u64_ops"] / 1e12, peaks["valu_exp_ops"] / 1e12,
                    peaks["lds_read_bytes"] / 1e12))
    if args.peaks:
        r = peaks
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
    progress("workload %s ready" % args.workload)
    attempts_per_step = work.attempts_per_sweep() * SWEEPS_PER_STEP
    timed = time_workload(binding, work, stream, args.steps, args.warmup, tier=args.tier,
                          autotune=not args.no_autotune, batch=False if args.class_launches else None)
    dt = timed["dt"]
    value = attempts_per_step * args.steps / (dt * 1e9)
    progress("timed %d graph-replayed steps in %.3f s: %.1f attempts/ns (direct launches: %.3f ms per step)"
             % (args.steps, dt, value, timed["direct_ms_per_step"]))
    roofline = roofline_of(args.workload, work, timed, args.tier, peaks)

    unbatched = None
    if not args.no_unbatched:
        unbatched = time_unbatched(binding, work, stream, args.unbatched_samples, args.unbatched_steps,
                                   tier=args.tier)
        unbatched["batched_over_unbatched"] = value / unbatched["value"]
        progress("unbatched: %.1f attempts/ns" % unbatched["value"])
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

    extra = None
    if not args.no_extra and args.workload == "L16_gauss" and args.tier == 0:
        extra = {}
        for name in EXTRA_WORKLOADS:
            w2 = W.config_workload(name, measure_start=0, measure_every=10)
            t2 = time_workload(binding, w2, stream, args.extra_steps, 1, autotune=not args.no_autotune)
            v2 = w2.attempts_per_sweep() * SWEEPS_PER_STEP * args.extra_steps / (t2["dt"] * 1e9)
            ub = time_unbatched(binding, w2, stream, 16, 1)
            extra[name] = {"workload": WORKLOAD_TEXT[name], "value": v2, "unit": "attempts/ns",
                           "steps": args.extra_steps, "ms_per_step": t2["ms_per_step"],
                           "engines": t2["engines"], "plan": t2["plan"],
                           "roofline": roofline_of(name, w2, t2, 0, peaks),
                           "unbatched": dict(ub, batched_over_unbatched=v2 / ub["value"])}
            progress("%s: %.1f attempts/ns, frac %.3f, unbatched %.1f"
                     % (name, v2, extra[name]["roofline"]["frac"], ub["value"]))
            del w2

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
                   "attempts_per_step": attempts_per_step, "plan": timed["plan"],
                   "tier": args.tier, "timed_path": "hipGraph replay of each 100-sweep chunk",
                   "direct_launch_ms_per_step": timed["direct_ms_per_step"],
                   "parallelism": "samples x chains across workgroups"},
        "unbatched": unbatched,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "other_workloads": extra,
        "peaks_measured": None if peaks is None else {
            "valu_xor_Tops": peaks["valu_xor_ops"] / 1e12, "valu_mad_u64_Tops": peaks["valu_mad_u64_ops"] / 1e12,
            "valu_exp_Tops": peaks["valu_exp_ops"] / 1e12, "lds_read_TBps": peaks["lds_read_bytes"] / 1e12,
            "hbm_copy_TBps": peaks["hbm_copy_bytes"] / 1e12},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
