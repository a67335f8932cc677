// ea_kernels.hip -- gfx950 kernels of the Edwards-Anderson Monte Carlo engine.
//
// LDS-resident tier (L <= 16).  One workgroup owns one (sample, chain) work
// item for a chunk of K sweeps: the chain's n_T walkers (int8 spins) and the
// sample's couplings (float32 or int8) are loaded into LDS once, then every
// sweep of the chunk -- two checkerboard half-sweeps of Metropolis updates
// (Methods: single-spin-flip Monte Carlo), the exact energy bookkeeping, the
// replica-exchange pass (Methods: parallel tempering) and, when due, a
// snapshot of the chain in slot order for the overlap measurement -- runs out
// of LDS.  Spins and maps go back to HBM once per chunk.
//
// The two chains of a sample only meet in the overlap q_i = s_i^a s_i^b
// (eq. 2), so they are independent work items; the measurement kernel
// combines their snapshots after the chunk.
#include "ea_device.hpp"
#include "ea_types.hpp"

namespace ea {

// Block-cooperative byte copy, 16 bytes at a time when both ends allow it.
__device__ __forceinline__ void block_copy(void *dst, const void *src, size_t bytes)
{
    const int T = blockDim.x, tid = threadIdx.x;
    if ((((uintptr_t)dst | (uintptr_t)src | bytes) & 15) == 0) {
        int4 *d = (int4 *)dst;
        const int4 *s = (const int4 *)src;
        for (size_t i = tid; i < bytes / 16; i += T) d[i] = s[i];
    } else {
        int8_t *d = (int8_t *)dst;
        const int8_t *s = (const int8_t *)src;
        for (size_t i = tid; i < bytes; i += T) d[i] = s[i];
    }
}

__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const int lo = __shfl_xor((int)(unsigned long long)v, m);
        const int hi = __shfl_xor((int)((unsigned long long)v >> 32), m);
        v += (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    }
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// One checkerboard half-sweep (parity p) over every walker of the chain.  A
// thread takes groups of four consecutive sublattice sites (one Philox call,
// word h&3 for site h) of one walker; sites of one parity never neighbour each
// other, so the updates of a half-sweep are independent.
template <int L, int JK>
__device__ __forceinline__ void half_sweep(const SweepArgs &A, const SampleDev &d, int r, int p,
                                           int64_t n, int8_t *S, const void *Jl, const int32_t *sow,
                                           int32_t *dM, int32_t *fl, long long *dEJ,
                                           const uint32_t *lut, const float *b32)
{
    constexpr int N = L * L * L, HALF = N / 2, G = HALF / 4, HL = L / 2;
    const int nT = d.n_T;
    const int T = blockDim.x, tid = threadIdx.x;
    const int total = nT * G;
    const uint32_t c1 = (uint32_t)(2 * n + p);
    const uint32_t c2base = (PURPOSE_METROPOLIS << 28) | (uint32_t)r;
    for (int base = 0; base < total; base += T) {
        const int idx = base + tid;
        const bool act = idx < total;
        const int w = act ? idx / G : -1;
        const int g = act ? idx - w * G : 0;
        int t = 0;
        int dEu = 0, dm = 0, nfl = 0;
        if (act) {
            t = sow[w];
            const u32x4 rw = philox4x32_10((uint32_t)g, c1, c2base | ((uint32_t)t << 1), d.sample_id,
                                           A.key0, A.key1);
            const uint32_t words[4] = {rw.x, rw.y, rw.z, rw.w};
            int8_t *Sp = S + (size_t)w * N + p * HALF;
            const int8_t *So = S + (size_t)w * N + (1 - p) * HALF;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int h = 4 * g + i;
                const int row = h / HL, j = h - row * HL;
                const int y = row % L, z = row / L;
                const int x = 2 * j + ((y + z + p) & 1);
                const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
                const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
                const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
                const int rowc = L * (y + L * z);
                const int hxp = (xp + rowc) >> 1, hxm = (xm + rowc) >> 1;
                const int hyp = (x + L * (yp + L * z)) >> 1, hym = (x + L * (ym + L * z)) >> 1;
                const int hzp = (x + L * (y + L * zp)) >> 1, hzm = (x + L * (y + L * zm)) >> 1;
                const int si = Sp[h];
                const int s0 = So[hxp], s1 = So[hxm], s2 = So[hyp], s3 = So[hym], s4 = So[hzp],
                          s5 = So[hzm];
                bool accept;
                int units;
                if constexpr (JK == 0) {
                    const float *Jp = (const float *)Jl + p * 3 * HALF;
                    const float *Jo = (const float *)Jl + (1 - p) * 3 * HALF;
                    // exact: every partial sum is a multiple of 2^-18 below 2^6
                    float SJ = Jp[h] * (float)s0;
                    SJ = SJ + Jo[hxm] * (float)s1;
                    SJ = SJ + Jp[HALF + h] * (float)s2;
                    SJ = SJ + Jo[HALF + hym] * (float)s3;
                    SJ = SJ + Jp[2 * HALF + h] * (float)s4;
                    SJ = SJ + Jo[2 * HALF + hzm] * (float)s5;
                    const float f = SJ + d.h32;
                    const float dE = (2.0f * (float)si) * f;
                    const float e = exp_ea32(-(b32[t] * dE));
                    accept = (dE <= 0.0f) | (u24_of(words[i]) < e);
                    units = (int)(SJ * 262144.0f);
                } else {
                    const int8_t *Jp = (const int8_t *)Jl + p * 3 * HALF;
                    const int8_t *Jo = (const int8_t *)Jl + (1 - p) * 3 * HALF;
                    const int SJ = Jp[h] * s0 + Jo[hxm] * s1 + Jp[HALF + h] * s2 +
                                   Jo[HALF + hym] * s3 + Jp[2 * HALF + h] * s4 +
                                   Jo[2 * HALF + hzm] * s5;
                    const float f = (float)SJ + d.h32;  // sign of SJ + h is exact
                    const bool down = si * f <= 0.0f;
                    const uint32_t thr = lut[(t * 2 + ((si + 1) >> 1)) * 7 + ((SJ + 6) >> 1)];
                    accept = down | (words[i] < thr);
                    units = SJ;
                }
                if (accept) {
                    Sp[h] = (int8_t)(-si);
                    dEu += 2 * si * units;
                    dm -= 2 * si;
                    nfl += 1;
                }
            }
        }
        // Per-walker energy, magnetisation and per-slot flip counts: integer
        // sums, so their order does not matter.
        const int w0 = __shfl(w, 0);
        if (__all(w == w0 || w < 0)) {
            if (w0 >= 0) {
                const long long se = wave_sum_i64((long long)dEu);
                const int pk = wave_sum_i32(nfl + dm * 65536);
                if ((tid & 63) == 0) {
                    const int sfl = pk & 0xFFFF;
                    atomicAdd((unsigned long long *)&dEJ[w0], (unsigned long long)se);
                    atomicAdd(&dM[w0], (pk - sfl) / 65536);
                    atomicAdd(&fl[sow[w0]], sfl);
                }
            }
        } else if (act) {
            atomicAdd((unsigned long long *)&dEJ[w], (unsigned long long)(long long)dEu);
            atomicAdd(&dM[w], dm);
            atomicAdd(&fl[t], nfl);
        }
    }
}

template <int L, int JK>
__device__ void run_item(const SweepArgs &A, const SampleDev &d, int r, char *smem)
{
    constexpr int N = L * L * L;
    const int nT = d.n_T;
    const int T = blockDim.x, tid = threadIdx.x;
    const LdsOff o = lds_offsets(L, nT, JK);
    int8_t *S = (int8_t *)(smem + o.spins);
    void *Jl = (void *)(smem + o.J);
    int32_t *was = (int32_t *)(smem + o.was), *sow = (int32_t *)(smem + o.sow);
    int32_t *Mw = (int32_t *)(smem + o.M), *dM = (int32_t *)(smem + o.dM);
    int32_t *fl = (int32_t *)(smem + o.fl), *sw = (int32_t *)(smem + o.sw);
    long long *EJ = (long long *)(smem + o.EJ), *dEJ = (long long *)(smem + o.dEJ);
    uint32_t *lut = (uint32_t *)(smem + o.lut);
    float *b32 = (float *)(smem + o.b32);
    double *b64 = (double *)(smem + o.b64);

    const size_t sbase = (size_t)d.spin_off + (size_t)r * nT * N;
    const int gi = 2 * d.slot_off + r * nT;
    block_copy(S, A.spins + sbase, (size_t)nT * N);
    block_copy(Jl, (const char *)A.J + (size_t)d.J_off * (JK == 0 ? 4 : 1),
               (size_t)3 * N * (JK == 0 ? 4 : 1));
    for (int i = tid; i < nT; i += T) {
        was[i] = A.was[gi + i];
        EJ[i] = A.EJ[gi + i];
        Mw[i] = A.M[gi + i];
        fl[i] = 0;
        sw[i] = 0;
        b32[i] = A.beta32[d.slot_off + i];
        b64[i] = A.beta[d.slot_off + i];
    }
    if (JK == 1)
        for (int i = tid; i < nT * 14; i += T) lut[i] = A.lut[(size_t)d.slot_off * 14 + i];
    __syncthreads();

    const double unit = JK == 0 ? 0x1p-18 : 1.0;
    const double hd = (double)d.h32;
    const int64_t n0 = A.state[0];
    const int64_t cnt0 = measurements_upto(n0, A.measure_every, A.measure_start);
    for (int it = 0; it < A.K; ++it) {
        const int64_t n = n0 + it;
        for (int i = tid; i < nT; i += T) {
            sow[was[i]] = i;
            dEJ[i] = 0;
            dM[i] = 0;
        }
        __syncthreads();
        half_sweep<L, JK>(A, d, r, 0, n, S, Jl, sow, dM, fl, dEJ, lut, b32);
        __syncthreads();
        half_sweep<L, JK>(A, d, r, 1, n, S, Jl, sow, dM, fl, dEJ, lut, b32);
        __syncthreads();
        for (int i = tid; i < nT; i += T) {
            EJ[i] += dEJ[i];
            Mw[i] += dM[i];
        }
        __syncthreads();
        // Replica exchange of neighbouring slots (t, t+1), t = n&1, n&1 + 2, ...
        for (int j = tid;; j += T) {
            const int t = (int)(n & 1) + 2 * j;
            if (t + 1 >= nT) break;
            const int w0 = was[t], w1 = was[t + 1];
            const double E0 = (double)EJ[w0] * unit - hd * (double)Mw[w0];
            const double E1 = (double)EJ[w1] * unit - hd * (double)Mw[w1];
            const double D = (b64[t] - b64[t + 1]) * (E0 - E1);
            bool acc = D >= 0.0;
            if (!acc) {
                const u32x4 q = philox4x32_10(0u, (uint32_t)n,
                                              (PURPOSE_EXCHANGE << 28) | ((uint32_t)t << 1) | (uint32_t)r,
                                              d.sample_id, A.key0, A.key1);
                acc = u53_of(q.x, q.y) < exp_ea64(D);
            }
            if (acc) {
                was[t] = w1;
                was[t + 1] = w0;
                sw[t] += 1;
            }
        }
        __syncthreads();
        // Snapshot for the overlap measurement, in slot order.
        const int64_t done = n + 1;
        if (A.measure_every > 0 && done > A.measure_start &&
            (done - A.measure_start) % A.measure_every == 0) {
            const int64_t f = measurements_upto(done, A.measure_every, A.measure_start) - cnt0 - 1;
            int8_t *dst = A.frames + f * A.frame_bytes + sbase;
            for (int t = 0; t < nT; ++t) block_copy(dst + (size_t)t * N, S + (size_t)was[t] * N, N);
            for (int t = tid; t < nT; t += T) {
                const int w = was[t];
                A.frameE[f * 2 * A.total_slots + gi + t] = (double)EJ[w] * unit - hd * (double)Mw[w];
            }
        }
    }
    __syncthreads();
    block_copy(A.spins + sbase, S, (size_t)nT * N);
    for (int i = tid; i < nT; i += T) {
        A.was[gi + i] = was[i];
        A.EJ[gi + i] = EJ[i];
        A.M[gi + i] = Mw[i];
        A.flips[gi + i] += fl[i];
        A.swaps[gi + i] += sw[i];
    }
    __syncthreads();
}

template <int JK>
__global__ void __launch_bounds__(1024) lds_sweep_kernel(SweepArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (int item = blockIdx.x; item < A.n_items; item += gridDim.x) {
        const int code = A.items[item];
        const SampleDev d = A.samples[code >> 1];
        const int r = code & 1;
        switch (d.L) {
        case 2: run_item<2, JK>(A, d, r, smem); break;
        case 4: run_item<4, JK>(A, d, r, smem); break;
        case 6: run_item<6, JK>(A, d, r, smem); break;
        case 8: run_item<8, JK>(A, d, r, smem); break;
        case 10: run_item<10, JK>(A, d, r, smem); break;
        case 12: run_item<12, JK>(A, d, r, smem); break;
        case 14: run_item<14, JK>(A, d, r, smem); break;
        case 16: run_item<16, JK>(A, d, r, smem); break;
        default: break;  // the host never schedules other sizes here
        }
    }
}

template __global__ void lds_sweep_kernel<0>(SweepArgs);
template __global__ void lds_sweep_kernel<1>(SweepArgs);

// ---------------------------------------------------------------------------
// Overlap measurement (eq. 2).  One workgroup per (sample, slot): for each
// snapshot frame of the chunk, in time order, form q_i = s_i^a s_i^b, the
// integer sums S0 = sum q_i and the plane sums P_f[c] = sum of q_i over sites
// with k_f . r = c (mod L) for the nine wave vectors, then
// q(k_f) = sum_c P_f[c] e^{2 pi i c / L} / N (summed in c order) and add to
// the binary64 accumulators of the slot in time order.
__device__ __forceinline__ int plane_coord(int f, int L, int x, int y, int z)
{
    int c;
    switch (f) {
    case 0: c = x; break;
    case 1: c = y; break;
    case 2: c = z; break;
    case 3: c = x + y; break;
    case 4: c = x - y; break;
    case 5: c = x + z; break;
    case 6: c = x - z; break;
    case 7: c = y + z; break;
    default: c = y - z; break;
    }
    c %= L;
    return c < 0 ? c + L : c;
}

__global__ void __launch_bounds__(256) measure_kernel(MeasureArgs A)
{
    __shared__ int P[NPLANE][MAX_L];
    __shared__ int S0;
    __shared__ double accs[NACC];
    __shared__ double re_f[NPLANE], im_f[NPLANE];
    const int gs = blockIdx.x;
    const int s = A.slot_sample[gs];
    const SampleDev d = A.samples[s];
    const int t = gs - d.slot_off;
    const int L = d.L, N = L * L * L, HALF = N / 2, HL = L / 2;
    const int tid = threadIdx.x, T = blockDim.x;
    int64_t nf;
    if (A.explicit_frames > 0) {
        nf = A.explicit_frames;
    } else {
        const int64_t n0 = A.state[0];
        nf = measurements_upto(n0 + A.K, A.measure_every, A.measure_start) -
             measurements_upto(n0, A.measure_every, A.measure_start);
    }
    if (nf <= 0) return;
    for (int i = tid; i < NACC; i += T) accs[i] = A.acc[(size_t)gs * NACC + i];
    const double Nd = (double)N;
    for (int64_t f = 0; f < nf; ++f) {
        for (int i = tid; i < NPLANE * MAX_L; i += T) (&P[0][0])[i] = 0;
        if (tid == 0) S0 = 0;
        __syncthreads();
        const int8_t *sa = A.frames + f * A.frame_bytes + d.spin_off + (size_t)t * N;
        const int8_t *sb = sa + (size_t)d.n_T * N;
        int s0 = 0;
        for (int idx = tid; idx < N; idx += T) {
            const int p = idx >= HALF, h = idx - p * HALF;
            const int row = h / HL, j = h - row * HL, y = row % L, z = row / L;
            const int x = 2 * j + ((y + z + p) & 1);
            const int q = (int)sa[idx] * (int)sb[idx];
            s0 += q;
#pragma unroll
            for (int fam = 0; fam < NPLANE; ++fam) atomicAdd(&P[fam][plane_coord(fam, L, x, y, z)], q);
        }
        s0 = wave_sum_i32(s0);
        if ((tid & 63) == 0) atomicAdd(&S0, s0);
        __syncthreads();
        if (tid < NPLANE) {
            const double *ct = A.costab + (size_t)L * MAX_L, *st = A.sintab + (size_t)L * MAX_L;
            double re = 0.0, im = 0.0;
            for (int c = 0; c < L; ++c) {
                re += (double)P[tid][c] * ct[c];
                im += (double)P[tid][c] * st[c];
            }
            re_f[tid] = re / Nd;
            im_f[tid] = im / Nd;
        }
        __syncthreads();
        if (tid < NPLANE) {
            const double re = re_f[tid], im = im_f[tid];
            accs[5 + 3 * tid] += re;
            accs[6 + 3 * tid] += im;
            accs[7 + 3 * tid] += re * re + im * im;
        } else if (tid == NPLANE) {
            const double q0 = (double)S0 / Nd;
            accs[0] += 1.0;
            accs[1] += q0;
            accs[2] += q0 * q0;
            accs[3] += (q0 * q0) * q0;
            accs[4] += (q0 * q0) * (q0 * q0);
            const double *E = A.frameE + f * 2 * A.total_slots + 2 * (size_t)d.slot_off;
            const double Ea = E[t], Eb = E[d.n_T + t];
            accs[32] += Ea;
            accs[33] += Ea * Ea;
            accs[34] += Eb;
            accs[35] += Eb * Eb;
        }
        __syncthreads();
    }
    for (int i = tid; i < NACC; i += T) A.acc[(size_t)gs * NACC + i] = accs[i];
}

__global__ void advance_kernel(int64_t *state, int64_t k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) state[0] += k;
}

// ---------------------------------------------------------------------------
// From-scratch energies E_J (exact integer units) and magnetisations of every
// walker of one (sample, chain) per workgroup; used to verify the incremental
// bookkeeping and to rebuild the state after ea_write_state.
template <int JK>
__global__ void __launch_bounds__(256) energy_kernel(const SampleDev *samples, const int32_t *items,
                                                    const int8_t *spins, const void *J, int64_t *EJ_out,
                                                    int32_t *M_out)
{
    __shared__ long long se;
    __shared__ int sm;
    const int code = items[blockIdx.x];
    const SampleDev d = samples[code >> 1];
    const int r = code & 1;
    const int L = d.L, N = L * L * L, HALF = N / 2, HL = L / 2;
    const int tid = threadIdx.x, T = blockDim.x;
    for (int w = 0; w < d.n_T; ++w) {
        if (tid == 0) {
            se = 0;
            sm = 0;
        }
        __syncthreads();
        const int8_t *Sw = spins + d.spin_off + ((size_t)r * d.n_T + w) * N;
        long long e = 0;
        int m = 0;
        for (int idx = tid; idx < N; idx += T) {
            const int p = idx >= HALF, h = idx - p * HALF;
            const int row = h / HL, j = h - row * HL, y = row % L, z = row / L;
            const int x = 2 * j + ((y + z + p) & 1);
            const int si = Sw[idx];
            const int xp = (x + 1) % L, yp = (y + 1) % L, zp = (z + 1) % L;
            const int nb[3] = {(xp + L * (y + L * z)) >> 1, (x + L * (yp + L * z)) >> 1,
                               (x + L * (y + L * zp)) >> 1};
            for (int dd = 0; dd < 3; ++dd) {
                const int sj = Sw[(1 - p) * HALF + nb[dd]];
                long long Ju;
                if (JK == 0)
                    Ju = (long long)(((const float *)J)[d.J_off + (size_t)p * 3 * HALF + dd * HALF + h] *
                                     262144.0f);
                else
                    Ju = ((const int8_t *)J)[d.J_off + (size_t)p * 3 * HALF + dd * HALF + h];
                e -= Ju * si * sj;
            }
            m += si;
        }
        e = wave_sum_i64(e);
        m = wave_sum_i32(m);
        if ((tid & 63) == 0) {
            atomicAdd((unsigned long long *)&se, (unsigned long long)e);
            atomicAdd(&sm, m);
        }
        __syncthreads();
        if (tid == 0) {
            const size_t gi = 2 * (size_t)d.slot_off + (size_t)r * d.n_T + w;
            EJ_out[gi] = se;
            M_out[gi] = sm;
        }
        __syncthreads();
    }
}

template __global__ void energy_kernel<0>(const SampleDev *, const int32_t *, const int8_t *, const void *,
                                          int64_t *, int32_t *);
template __global__ void energy_kernel<1>(const SampleDev *, const int32_t *, const int8_t *, const void *,
                                          int64_t *, int32_t *);

// Snapshot of the current state (slot order) into frame 0, for an immediate
// measurement.  One workgroup per (sample, chain).
__global__ void __launch_bounds__(256) snapshot_kernel(const SampleDev *samples, const int32_t *items,
                                                      const int8_t *spins, const int32_t *was,
                                                      const int64_t *EJ, const int32_t *M, int jkind,
                                                      int8_t *frame, double *frameE)
{
    const int code = items[blockIdx.x];
    const SampleDev d = samples[code >> 1];
    const int r = code & 1;
    const size_t N = (size_t)d.L * d.L * d.L;
    const size_t sbase = (size_t)d.spin_off + (size_t)r * d.n_T * N;
    const int gi = 2 * d.slot_off + r * d.n_T;
    for (int t = 0; t < d.n_T; ++t) block_copy(frame + sbase + t * N, spins + sbase + (size_t)was[gi + t] * N, N);
    const double unit = jkind == 0 ? 0x1p-18 : 1.0;
    for (int t = threadIdx.x; t < d.n_T; t += blockDim.x) {
        const int w = was[gi + t];
        frameE[gi + t] = (double)EJ[gi + w] * unit - (double)d.h32 * (double)M[gi + w];
    }
}

// Disorder averages per slot over the samples of one lattice size and ladder
// length (eqs. 3-6).  Single workgroup; thread t handles slot t and sums over
// samples in sample order.
__global__ void finalize_kernel(const SampleDev *samples, int S, int L, int nT, const double *acc,
                                double *out)
{
    const int t = threadIdx.x;
    if (t >= nT) return;
    double D[NACC];
    for (int j = 0; j < NACC; ++j) D[j] = 0.0;
    int cnt = 0;
    for (int s = 0; s < S; ++s) {
        const SampleDev d = samples[s];
        if (d.L != L || d.n_T != nT) continue;
        const double *a = acc + ((size_t)d.slot_off + t) * NACC;
        for (int j = 0; j < NACC; ++j) D[j] += a[j] / a[0];
        ++cnt;
    }
    double *o = out + (size_t)t * 11;
    o[10] = (double)cnt;
    if (cnt == 0) return;
    for (int j = 0; j < NACC; ++j) D[j] /= (double)cnt;
    const double N = (double)L * L * L;
    const double q1 = D[1], q2 = D[2], q3 = D[3], q4 = D[4], Q = q1;
    const double c2 = q2 - 2.0 * Q * q1 + Q * Q;
    const double c4 = q4 - 4.0 * Q * q3 + 6.0 * Q * Q * q2 - 4.0 * Q * Q * Q * q1 + Q * Q * Q * Q;
    double chi[NPLANE];
    for (int f = 0; f < NPLANE; ++f) {
        const double re = D[5 + 3 * f], im = D[6 + 3 * f];
        chi[f] = N * (D[7 + 3 * f] - (re * re + im * im));
    }
    const double chi0 = N * (q2 - q1 * q1);
    const double chik = (chi[0] + chi[1] + chi[2]) / 3.0;
    const double chik2 = (chi[3] + chi[4] + chi[5] + chi[6] + chi[7] + chi[8]) / 6.0;
    o[0] = q1;
    o[1] = chi0;
    o[2] = chik;
    o[3] = chik2;
    o[4] = 0.5 * (3.0 - c4 / (c2 * c2));
    o[5] = sqrt(chi0 / chik - 1.0) / (2.0 * sin(3.141592653589793 / (double)L));
    o[6] = chik / chik2;
    o[7] = chi0 / chik;
    o[8] = D[32];
    o[9] = D[34];
}

}  // namespace ea
