/*
 * ea.h -- C ABI of the MI355X (gfx950) engine for Metropolis Monte Carlo with
 * parallel tempering on the three-dimensional Edwards-Anderson spin glass in a
 * uniform field (arXiv:1403.4560).
 *
 * The model is the Hamiltonian of eq. 1, H = -sum_<ij> J_ij S_i S_j - h sum_i S_i,
 * on a periodic simple cubic lattice of N = L^3 Ising spins (Methods).  Each
 * disorder sample ("sample") is simulated as two independent replicas
 * ("chains" a and b) at each of N_T temperatures, coupled only by parallel
 * tempering within a chain (Methods, parallel tempering paragraph).  The
 * library measures the two-replica overlap q(k) of eq. 2 at k = 0, at the three
 * axis vectors (2pi/L)e_d and at the six images of (2pi/L, 2pi/L, 0), and
 * accumulates the moments from which eqs. 3-6 (Binder ratio, chi(k), xi_L,
 * R12) follow (ea_finalize).
 *
 * Numeric contract (every result is bit-reproducible; see the oracle tests):
 *   site i = x + L(y + Lz), parity p = (x+y+z)&1, sublattice index h = i>>1;
 *   bond J_d[i] joins site i and site i + e_d (periodic), d = 0,1,2 = x,y,z.
 *   A sweep is: every parity-0 site of every walker, then every parity-1
 *   site (Metropolis, "checkerboard"), then one replica-exchange pass per
 *   chain over pairs (t,t+1) with t = n&1, n&1+2, ..., then a measurement if
 *   one is due.  Random numbers come from Philox4x32-10 (Salmon et al., SC'11)
 *   keyed by seed and addressed by (h>>2, 2n+p, (purpose<<28)|(t<<1)|r,
 *   sample_id); they depend on the temperature slot t, never on where a
 *   walker's spins live, so results do not depend on the launch plan.
 *   Local fields and the acceptance test are binary32 with an in-house
 *   exponential (exact on the 2^-18 coupling grid); energies are exact
 *   (integer units) and exchange probabilities and all accumulators binary64.
 *
 * Conventions for every entry point:
 *   - returns EA_OK (0) or a negative ea_status; no C++ exception crosses.
 *   - on failure, ea_last_error() returns a thread-local message.
 *   - pointers named *_host are host memory owned by the caller; the library
 *     copies what it needs before returning (create, write_state) or fills
 *     caller-allocated buffers of the documented size (measure, read_state).
 *   - device memory is owned by the ensemble and freed by ea_destroy.
 *   - after EA_EDEVICE the handle rejects every call but ea_destroy
 *     (EA_ESTATE).  A handle is not thread-safe.
 */
#ifndef EA_H
#define EA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ea_ensemble ea_ensemble;

typedef enum {
    EA_OK = 0,
    EA_EINVAL = -1,       /* invalid argument (message says which)              */
    EA_ENOMEM = -2,       /* device or host allocation failed                    */
    EA_EDEVICE = -3,      /* a HIP call failed; the handle is now unusable      */
    EA_ESTATE = -4,       /* handle unusable, or tracked state inconsistent     */
    EA_EUNSUPPORTED = -5  /* valid but not supported (e.g. odd L)               */
} ea_status;

enum { EA_J_GAUSS_F32 = 0, EA_J_PM1_I8 = 1 };

/* Accumulators per (sample, slot), binary64, summed over measurements:
 *   [0] n            [1..4] sum of q0, q0^2, q0^3, q0^4 (q0 = q(k=0), eq. 2)
 *   [5+3f], [6+3f], [7+3f]: sum of Re q(k_f), Im q(k_f), |q(k_f)|^2 for
 *     f = 0,1,2: k = (2pi/L) e_x, e_y, e_z;
 *     f = 3..8: k = (2pi/L) (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1),
 *     (0,1,-1)
 *   [32], [33]: sum of E, E^2 of chain a's walker at the slot;
 *   [34], [35]: the same for chain b.                                      */
enum { EA_NACC = 36, EA_NPLANE = 9 };

/* Input description for ea_create_ensemble.  All arrays are host memory in
 * sample-concatenated order; n_T and L may differ between samples. */
typedef struct {
    int32_t n_samples;           /* S >= 1                                      */
    const uint32_t *sample_id;   /* [S] Philox address word 3; NULL => 0..S-1   */
    const int32_t *L;            /* [S] even, 2 <= L <= 32                      */
    const int32_t *n_temps;      /* [S] 1 <= n_T <= 64                          */
    const double *beta;          /* concat [S][n_T]: finite, > 0, non-decreasing;
                                    <= 2^20 with Gaussian couplings (the
                                    acceptance shortcut's error bound) */
    const float *h;              /* [S] uniform field, finite                    */
    int32_t jkind;               /* EA_J_GAUSS_F32 or EA_J_PM1_I8                */
    const void *J;               /* concat [S][3][N]: float on the 2^-18 grid
                                    with |J| < 8, or int8 +-1                    */
    const int8_t *spins0;        /* concat [S][2][n_T][N], values +-1, walker w
                                    starts at slot w                             */
    uint64_t seed;               /* Philox key: k0 = low, k1 = high 32 bits     */
    int32_t measure_every;       /* m >= 1, or 0 = never measure                */
    int64_t measure_start;       /* measure after sweep n iff n+1 > start and
                                    (n+1-start) % m == 0                         */
    int32_t tier;                /* EA_TIER_AUTO: chains that fit LDS stay
                                    there (int8 spins for L <= 16; one bit per
                                    spin for +-1 couplings at L = 8, 16, 32),
                                    larger ones in HBM (L divisible by 8);
                                    EA_TIER_HBM: every sample whose L is
                                    divisible by 8 runs HBM-resident;
                                    EA_TIER_BYTES: as AUTO without the
                                    one-bit engine; EA_TIER_SITE: every
                                    LDS-resident sample on the one-site-per-
                                    thread engine.  Results are identical. */
} ea_desc;

enum { EA_TIER_AUTO = 0, EA_TIER_HBM = 1, EA_TIER_BYTES = 2, EA_TIER_SITE = 3 };

/* Launch plan.  Every plan gives bit-identical results. */
typedef struct {
    int32_t chunk;      /* sweeps per persistent launch (>= 1)                  */
    int32_t threads;    /* threads per workgroup of the site engine's own
                           launches: 256, 512 or 1024                           */
    int32_t use_graph;  /* 1: replay each chunk from a captured hipGraph       */
    int32_t batch;      /* 1: the lattice-size classes of the group engine,
                           the L = 8 row engine and the L <= 4 site engine
                           run as one launch per chunk (one workgroup per
                           unit, units ordered longest first, each unit up to
                           P items of one class run side by side by P teams
                           of a workgroup; P per class is chosen by
                           ea_autotune); 0: one launch per class.  Default 1
                           when two or more such classes exist.             */
} ea_plan;

/* Create an ensemble from a description, copy it to the device and bind it
 * to a HIP stream (NULL: the null stream).  *out is NULL on failure.
 * Errors: EA_EINVAL for a malformed description (odd or out-of-range L,
 * spins not +-1, couplings off their alphabet, bad beta, bad m/start),
 * EA_ENOMEM, EA_EDEVICE. */
ea_status ea_create_ensemble(const ea_desc *desc, void *hip_stream, ea_ensemble **out);
/* Lattice sizes: every even L in [2, 16] runs LDS-resident (one workgroup per
 * (sample, chain) holding the chain for a chunk of sweeps), and so does L = 32
 * with +-1 couplings when the chain fits LDS at one bit per spin (n_T <= 32);
 * other L in {24, 32} (and 8, 16 under EA_TIER_HBM) run HBM-resident (four
 * launches per sweep).  Other sizes above 16 return EA_EUNSUPPORTED. */

/* Advance every sample by n_sweeps sweeps (half-sweep p=0, half-sweep p=1,
 * replica exchange, measurement if due; Methods).  Asynchronous on the bound
 * stream; n_sweeps >= 0.  sweep_pt(a) then sweep_pt(b) equals sweep_pt(a+b)
 * bit for bit. */
ea_status ea_sweep_pt(ea_ensemble *ens, int64_t n_sweeps);

/* The same computation, launched one sample at a time (two workgroups per
 * launch) serially on the bound stream: the unbatched comparator.  Results
 * are bit-identical to ea_sweep_pt. */
ea_status ea_sweep_pt_unbatched(ea_ensemble *ens, int64_t n_sweeps);

/* Copy the accumulators and counters to the host and synchronize.
 * flags & EA_MEASURE_NOW first measures the current state once.
 * acc_host   [S][n_T][36] (layout above; may be NULL)
 * flips_host [S][2][n_T] accepted spin flips per (sample, chain, slot)
 * swaps_host [S][2][n_T] accepted exchanges of pair (t, t+1) at index t      */
enum { EA_MEASURE_NOW = 1 };
ea_status ea_measure(ea_ensemble *ens, int32_t flags, double *acc_host,
                     int64_t *flips_host, int64_t *swaps_host);

/* Copy the state to the host and synchronize.  Any pointer may be NULL.
 * spins_host      [S][2][n_T][N] int8 in slot order (index t holds the walker
 *                 at slot t), natural site order
 * walker_at_slot  [S][2][n_T]
 * E_host          [S][2][n_T] total energy (eq. 1) of the walker at each slot
 * sweep           sweeps completed                                         */
ea_status ea_read_state(ea_ensemble *ens, int8_t *spins_host, int32_t *walker_at_slot,
                        double *E_host, int64_t *sweep);

/* Replace the state (resume from a checkpoint): spins in slot order as
 * returned by ea_read_state ([S][2][n_T][N], host, copied), the walker at
 * each slot as returned by ea_read_state ([S][2][n_T], each chain's entries a
 * permutation of 0 .. n_T-1; EA_EINVAL otherwise), or NULL to put walker t at
 * slot t (walker labels never change a later result: random numbers are
 * keyed by slot), and the sweep counter.  Energies and magnetisations are
 * recomputed on the device.  Accumulators and counters are left alone.
 * Synchronizing. */
ea_status ea_write_state(ea_ensemble *ens, const int8_t *spins_host, const int32_t *walker_at_slot, int64_t sweep);

/* Load accumulators and counters (any NULL is left alone); layouts as in
 * ea_measure. */
ea_status ea_load_accumulators(ea_ensemble *ens, const double *acc_host,
                               const int64_t *flips_host, const int64_t *swaps_host);

/* Zero accumulators and counters. */
ea_status ea_reset_accumulators(ea_ensemble *ens);

/* Recompute every walker's energy from its spins on the device and compare
 * with the incrementally tracked value.  *mismatches = number of walkers
 * that differ (0 for a consistent state).  Synchronizing. */
ea_status ea_check_energies(ea_ensemble *ens, int64_t *mismatches);

/* Disorder averages per temperature slot over the selected samples of one
 * system (eqs. 3-6), computed on the device from the accumulators.  The
 * overline of eqs. 3-6 averages over disorder realizations of one model, so a
 * selection must be one system: samples[0..n_samples-1] are distinct indices
 * into the ensemble that share the lattice size, the temperature ladder (every
 * beta, bit for bit) and the field; samples == NULL selects every sample
 * (n_samples is then ignored).  A disorder average is the exact sum of the
 * per-sample thermal means (accumulated sum / number of measurements), rounded
 * once to binary64 and divided by the count, so it does not depend on the
 * order of the samples; each observable is then evaluated in the order its
 * formula is written.  out_host [n_T][EA_NOBS] binary64 (caller-owned),
 * columns in ea_obs order.  EA_EINVAL for an empty, out-of-range, repeated or
 * mixed selection (different L, ladder or field).  Synchronizing. */
enum {
    EA_OBS_Q = 0,        /* [<q(0)>]                                          */
    EA_OBS_CHI0,         /* chi(0) = N([<q^2>] - [<q>]^2)            eq. 4     */
    EA_OBS_CHIKMIN,      /* chi at |k| = 2pi/L, mean of three axes   eq. 4     */
    EA_OBS_CHIK2,        /* chi at (2pi/L)(1,1,0), mean of six images          */
    EA_OBS_BINDER,       /* g of eq. 3, moments centred on [<q(0)>]            */
    EA_OBS_XI,           /* xi_L of eq. 5                                      */
    EA_OBS_R12,          /* chi(k1)/chi(k2) of eq. 6                           */
    EA_OBS_RATIO,        /* chi(0)/chi(kmin)                                   */
    EA_OBS_EA,           /* [<E>] chain a                                      */
    EA_OBS_EB,           /* [<E>] chain b                                      */
    EA_OBS_NSAMP,        /* number of samples averaged                         */
    EA_NOBS
};
ea_status ea_finalize(ea_ensemble *ens, const int32_t *samples, int32_t n_samples, double *out_host);

/* The same observables with their statistical errors from the disorder
 * average (Methods, last paragraph: the error comes from the finite number of
 * realizations), over a selection as for ea_finalize: leave-one-sample-out
 * jackknife on the device.  Replicate s uses the exact sum of the other
 * samples' thermal means rounded once and divided by the count less one; the
 * error is sqrt((S-1)/S * sum_s (O_s - Obar)^2) with Obar and the sum of
 * squares again exact sums rounded once.  out_mean and out_err [n_T][EA_NOBS]
 * binary64 (caller-owned); out_mean equals ea_finalize's result, out_err holds
 * the jackknife standard errors (0 in the EA_OBS_NSAMP column).  EA_EINVAL as
 * for ea_finalize, or if fewer than two samples are selected.
 * Synchronizing. */
ea_status ea_finalize_jackknife(ea_ensemble *ens, const int32_t *samples, int32_t n_samples, double *out_mean,
                                double *out_err);

/* ea_finalize_jackknife for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and errors, bit-identical to
 * ea_finalize_jackknife, but no device or host allocation.  The jackknife
 * replicates (n_temps x selected samples x 10 doubles) go to a fixed scratch
 * array of 8 MiB that every device the library runs on holds until the
 * process ends (its address is looked up when an ensemble is created on that
 * device); EA_EINVAL if n_temps x samples exceeds 104857.  Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be serialized by the caller.
 * EA_EDEVICE if the scratch address could not be obtained.  Synchronizing. */
ea_status ea_finalize_jackknife_noalloc(ea_ensemble *ens, const int32_t *samples, int32_t n_samples,
                                        double *out_mean, double *out_err);

/* Launch plan (see ea_plan); EA_EINVAL for values out of range. */
ea_status ea_set_plan(ea_ensemble *ens, const ea_plan *plan);
ea_status ea_get_plan(const ea_ensemble *ens, ea_plan *plan);

/* Time candidate plans on a copy of the state (the ensemble's state and
 * accumulators are restored afterwards) and keep the fastest: the teams per
 * batch workgroup of every batch class (coordinate descent, class by class),
 * the batch launch against one launch per class, and the workgroup size of
 * the site engine's own launches.  If the environment variable EA_TUNE_CACHE
 * names a file, a plan stored there under this ensemble's signature (device,
 * coupling kind and launch classes) is applied without timing, and a newly
 * tuned plan is stored.  The chunk length and graph use are left alone.
 * Synchronizing.  trial_sweeps >= 1. */
ea_status ea_autotune(ea_ensemble *ens, int32_t trial_sweeps);

/* The layout of the batch launch (ea_plan.batch): one entry per launch class
 * (a lattice size and engine, in launch order).  *n_classes receives the
 * count; class_L, class_engine (ea_engine values) and teams [n_classes] may
 * be NULL.  teams[c] = work items of class c that one batch workgroup runs
 * side by side (1, 2, 4 or 8 teams of 512/teams threads), 0 for a class the
 * batch launch does not take (one-bit, HBM-resident, and row-engine L = 16
 * classes keep their own launches).  With the batch launch off, a group-engine
 * class runs its own launch with workgroups of the same team size.
 * signature (17 bytes, may be NULL) receives the key under which ea_autotune
 * caches this ensemble's plan. */
ea_status ea_get_batch_plan(const ea_ensemble *ens, int32_t *n_classes, int32_t *class_L, int32_t *class_engine,
                            int32_t *teams, char *signature);

/* Set teams per batch workgroup for every class (layout as returned by
 * ea_get_batch_plan; 0 for classes the batch launch does not take).
 * EA_EINVAL if a value is not possible for its class (teams too small for the
 * class's items, or their LDS frames beyond one workgroup's).  Results are
 * unchanged; only the launch shape is.  Synchronizing. */
ea_status ea_set_batch_plan(ea_ensemble *ens, const int32_t *teams);

/* Kernel timing on the bound stream: when enabled, the sweep kernels of every
 * chunk (one launch, or one per launch class; the measurement launch
 * excluded) are bracketed by a pair of HIP events; ea_kernel_time returns the
 * summed duration in milliseconds and the number of chunks timed since it was
 * enabled (it synchronizes).  Graph replay is bypassed while timing is on. */
ea_status ea_set_timing(ea_ensemble *ens, int32_t enable);
ea_status ea_kernel_time(ea_ensemble *ens, double *ms_total, int64_t *launches);

/* Block the host until all work on the bound stream has finished. */
ea_status ea_synchronize(ea_ensemble *ens);

/* Sizes: samples, total slots (sum n_T), device bytes held. */
ea_status ea_query(const ea_ensemble *ens, int32_t *n_samples, int64_t *total_slots,
                   int64_t *device_bytes);

/* Device bytes of the persistent buffers an ensemble created from desc would
 * hold (samples, couplings, spins, temperatures, walker maps, energies,
 * counters, accumulators, tables), laid out as one arena of 256-byte aligned
 * slices: the size of the caller memory ea_bind_buffers takes.  The snapshot
 * frames (sized by the plan's chunk) and the scratch of ea_check_energies are
 * not part of it and stay library-owned.  Validates desc as
 * ea_create_ensemble does and asks the current device for its LDS size (which
 * decides the engines); allocates nothing.  EA_EDEVICE without a device. */
ea_status ea_query_sizes(const ea_desc *desc, size_t *device_bytes);

/* Move the ensemble's persistent buffers into caller-owned device memory, for
 * callers that account memory themselves (a torch tensor, say).
 * device_ptrs[0] is the arena: arena_bytes (at least ea_query_sizes bytes) of
 * device memory of the ensemble's device, 256-byte aligned, left untouched by
 * the caller while the ensemble lives.  The current contents are copied over
 * (synchronizing the stream) and the library's own buffers freed; from then on
 * the library reads and writes the arena and never frees it (ea_destroy
 * leaves it to the caller).  Results are the same as without binding.
 * EA_EINVAL for a NULL, misaligned or too small arena (checked against the
 * allocation that holds it), EA_ESTATE if already bound. */
ea_status ea_bind_buffers(ea_ensemble *ens, void *const *device_ptrs, size_t arena_bytes);

/* The engine that runs each sample's sweeps (chosen at creation from L, n_T,
 * the coupling kind, the field, the LDS size and the tier option).
 * engines_host [S] (caller-owned) receives one ea_engine value per sample. */
enum {
    EA_ENGINE_SITE = 0,   /* LDS, one site of one walker per thread step        */
    EA_ENGINE_ROW = 1,    /* LDS, int8x4 words of one walker (Gaussian, 8, 16)  */
    EA_ENGINE_GROUP = 2,  /* LDS, int8x4 words of one site of four walkers      */
    EA_ENGINE_BITS = 3,   /* LDS, one bit per spin (+-1, L = 8, 16, 32)         */
    EA_ENGINE_HBM = 4     /* HBM-resident, four launches per sweep              */
};
ea_status ea_query_engines(const ea_ensemble *ens, int32_t *engines_host);

/* Device self-check of the acceptance shortcut used by the sweep kernels.
 * The kernels form an exponent y estimating x log2 e for x = -fl32(beta dE)
 * (within a relative 2^-21 plus 2^-20, from their roundings), a = 2^y with the
 * hardware exponential, and the gap g = fl32(fl32(w) - a 2^32) for the random
 * word w; g < -8192 accepts and g > 8192 rejects without evaluating the
 * in-house exp_ea32, any other word takes the exact test (x >= 0 or
 * U 2^-24 < exp_ea32(x), U = w >> 8).  This call checks, over every non-NaN
 * binary32 x (4.3e9 values) and at both ends of that range of y, the bounds on
 * a that make both shortcuts decide as the exact test would for every w: for
 * x <= 0 that a 2^32 lies within 8192 - 384 below and 8192 - 128 above
 * exp_ea32(x) 2^32 (exp_ea32 = 0 below -86), for x > 0 that a 2^32 >=
 * 2^32 - 8192 + 384; and that the hardware exponential is monotone over every
 * binary32 input.  *violations must be 0; *max_rel_dev is the largest
 * |a/exp_ea32(x) - 1| seen on [-86, 0].  Synchronizing; uses the current
 * device. */
ea_status ea_verify_exp_bracket(int64_t *violations, double *max_rel_dev);

/* Check of the replica-exchange shortcut (Methods: parallel tempering; the
 * acceptance min(1, e^D) as u53 < exp_ea64(D)).  For D < 0 the kernels decide
 * from a = 2^y, y = fl32(D log2 e), the hardware exponential: D < -40 rejects
 * (u53 >= 2^-53 > exp_ea64(D)) unless u53 = 0; for -40 <= D < 0,
 * u53 < a (1 - 2^-16) accepts and u53 > a (1 + 2^-16) rejects; anything else
 * evaluates exp_ea64.  The rounding of y moves a by at most a relative
 * 1.32e-6 (|y| < 58, half an ulp of 2^-18); this call checks, over every
 * binary32 y in [-58, 0] (1.1e9 values), the remaining bounds: the hardware
 * exponential within a relative 2^-22 of 2^y and exp_ea64(y) within 2^-49 of
 * e^y, so that a / exp_ea64(D) stays within 1 +- 1.7e-6 and both shortcuts
 * decide as the exact test would; it also compares the kernels' decision with
 * the exact test for D = 1.5 y (down to -87) at uniforms spread across the
 * margin, at u = 0 and at the largest u.  *violations must be 0;
 * *max_rel_dev is the largest relative deviation of the hardware exponential
 * seen.  Synchronizing; uses the current device. */
ea_status ea_verify_exchange_bracket(int64_t *violations, double *max_rel_dev);

/* Microbenchmarks of the rates the kernels' rooflines are priced against, on
 * the current device (about a second; synchronizing; allocates and frees
 * 2 GiB for the copy).  rates_host[6] (caller-owned) receives, per second:
 * [0] v_xor_b32 lane-operations, [1] v_mad_u64_u32 lane-operations,
 * [2] v_mul_hi_u32 lane-operations (sixteen independent chains per lane, eight
 * waves per SIMD), [3] LDS bytes read (16-byte reads, no bank conflicts),
 * [4] HBM bytes read plus written by a 1 GiB device copy, [5] v_exp_f32
 * lane-operations (as [0]). */
ea_status ea_measure_peaks(double *rates_host);

void ea_destroy(ea_ensemble *ens);
const char *ea_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EA_H */
