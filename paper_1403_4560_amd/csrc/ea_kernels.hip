// ea_kernels.hip -- gfx950 kernels of the Edwards-Anderson Monte Carlo engine.
//
// LDS-resident tier (L <= 16).  One workgroup owns one (sample, chain) work
// item for a chunk of K sweeps: the chain's n_T walkers (int8 spins) and the
// sample's couplings are loaded into LDS once, then every sweep of the chunk --
// two checkerboard half-sweeps of Metropolis updates (Methods: single-spin-flip
// Monte Carlo), the exact energy bookkeeping, the replica-exchange pass
// (Methods: parallel tempering) and, when due, a snapshot of the chain in slot
// order for the overlap measurement -- runs out of LDS.  Spins and maps go back
// to HBM once per chunk.
//
// The two chains of a sample only meet in the overlap q_i = s_i^a s_i^b
// (eq. 2), so they are independent work items; the measurement kernel
// combines their snapshots after the chunk.
//
// Two half-sweep engines share that frame here:
//  * row engine (L = 8, 16; Gaussian couplings): a thread owns one walker and
//    one (x-word, y) column and walks z; it works on 4 sites at once (one int8x4
//    word = one Philox call), keeps couplings as integer 2^-18 units and the
//    walker's energy/flip tallies in registers for the whole sweep;
//  * site engine (any even L <= 16, either coupling kind; chains too small for
//    the group engine): a thread takes a 4-site group of any walker and updates
//    its sites one by one.
// The group engine (ea_group.hip: one word = one site of four walkers) and the
// one-bit engine (ea_bits.hip: +-1 couplings) use the same frame with their
// own LDS layouts.  This file also holds the HBM-resident tier, the overlap
// measurement and the setup and check kernels (finalize: ea_finalize.hip).
#include "ea_device.hpp"
#include "ea_item.hpp"
#include "ea_row.hpp"
#include "ea_types.hpp"
#include "ea_update.hpp"

namespace ea {

// One kernel per (engine, L, coupling kind).  VAR only separates the symbol
// of the one-sample-per-launch comparator from the batched launch in
// profiles; the code is identical.
template <int L, int JK, int VAR>
__global__ void __launch_bounds__(1024) site_sweep_kernel(SweepArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (int item = blockIdx.x; item < A.n_items; item += gridDim.x) {
        const int code = A.items[item];
        run_item<L, JK, false>(A, A.samples[code >> 1], code & 1, smem);
    }
}

// L = 8 chains are small (two waves for 16 walkers), so their workgroups are
// held to 128 VGPRs to keep four waves per SIMD resident.
template <int L, int VAR>
__global__ void __launch_bounds__(ROW_MAX_THREADS, L == 8 ? 4 : 1) row_sweep_kernel(SweepArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (int item = blockIdx.x; item < A.n_items; item += gridDim.x) {
        const int code = A.items[item];
        run_item<L, 0, true>(A, sample_of_item(A.samples, code >> 1), code & 1, smem);
    }
}

#define EA_SITE(Lv)                                               \
    template __global__ void site_sweep_kernel<Lv, 0, 0>(SweepArgs); \
    template __global__ void site_sweep_kernel<Lv, 1, 0>(SweepArgs); \
    template __global__ void site_sweep_kernel<Lv, 0, 1>(SweepArgs); \
    template __global__ void site_sweep_kernel<Lv, 1, 1>(SweepArgs);
EA_SITE(2)
EA_SITE(4)
EA_SITE(6)
EA_SITE(8)
EA_SITE(10)
EA_SITE(12)
EA_SITE(14)
EA_SITE(16)
#undef EA_SITE
template __global__ void row_sweep_kernel<8, 0>(SweepArgs);
template __global__ void row_sweep_kernel<8, 1>(SweepArgs);
template __global__ void row_sweep_kernel<16, 0>(SweepArgs);
template __global__ void row_sweep_kernel<16, 1>(SweepArgs);

// ---------------------------------------------------------------------------
// HBM-resident tier (chains too large for LDS, e.g. L = 32).  Spins stay in
// HBM in the same sublattice layout; each sweep is four launches: half-sweep
// p = 0, half-sweep p = 1, exchange, snapshot.  A half-sweep workgroup takes a
// tile of up to 1024 int8x4 words of one walker (4 per thread); energy,
// magnetisation and flip tallies are reduced per workgroup and added to the
// walker's per-sweep change with integer atomics (order-free).  Blocks of one
// sample are kept on one XCD (blocks are dealt to the 8 XCDs round-robin) so
// the sample's couplings stay in that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int nb8 = nb & ~7;
    return b < nb8 ? (b & 7) * (nb8 >> 3) + (b >> 3) : b;
}

template <int W>
__device__ __forceinline__ void block_sum3(long long &a, int &b, int &c)
{
    __shared__ long long sa[W / 64];
    __shared__ int sb[W / 64], sc[W / 64];
    a = wave_sum_i64(a);
    b = wave_sum_i32(b);
    c = wave_sum_i32(c);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[wv] = a;
        sb[wv] = b;
        sc[wv] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < W / 64; ++i) {
            a += sa[i];
            b += sb[i];
            c += sc[i];
        }
    }
}

template <int L, int JK, int VAR>
__global__ void __launch_bounds__(256) hbm_half_kernel(SweepArgs A)
{
    constexpr int N = L * L * L, HALF = N / 2, WPR = L / 8, HL = L / 2, G = HALF / 4;
    constexpr int TILE = G < 1024 ? G : 1024, TPW = (G + TILE - 1) / TILE;
    __shared__ uint32_t thr[14];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int wi = b / TPW, tile = b - wi * TPW;
    if (wi >= A.n_walkers) return;
    const int code = A.walkers[wi];
    const SampleDev d = A.samples[code >> 7];
    const int r = (code >> 6) & 1, w = code & 63;
    const int nT = d.n_T, gi = 2 * d.slot_off + r * nT;
    const int t = A.sow[gi + w];
    const int p = A.p;
    const int64_t n = A.state[0] + A.it;
    const int tid = threadIdx.x;
    if (JK == 1 && tid < 14) thr[tid] = A.lut[((size_t)d.slot_off + t) * 14 + tid];
    __syncthreads();
    uint8_t *Sw = (uint8_t *)A.spins + d.spin_off + ((size_t)r * nT + w) * N;
    uint8_t *own = Sw + p * HALF;
    const uint8_t *oth = Sw + (1 - p) * HALF;
    const uint32_t c1 = (uint32_t)(2 * n + p);
    const uint32_t c2 = (PURPOSE_METROPOLIS << 28) | ((uint32_t)t << 1) | (uint32_t)r;
    const float b32 = A.beta32[d.slot_off + t];
    const float cp = two_beta_log2e(b32);
    const float ka = cp * 0x1p-18f, kb = cp * (d.h32 - (float)d.hgrid * 0x1p-18f);
    int accE = 0, bf = 0, bd = 0;
    for (int j = 0; j < (TILE + 255) / 256; ++j) {
        const int g = tile * TILE + j * 256 + tid;
        if (j * 256 + tid >= TILE || g >= G) break;
        const int k = g % WPR, row = g / WPR, y = row % L, z = row / L;
        const int eps = (y + z + p) & 1;
        const int kx = eps ? (k + 1) % WPR : (k + WPR - 1) % WPR;
        const int yp = (y + 1) % L, ym = (y + L - 1) % L, zp = (z + 1) % L, zm = (z + L - 1) % L;
        const int g_x = row * WPR + kx;
        const int g_yp = (yp + L * z) * WPR + k, g_ym = (ym + L * z) * WPR + k;
        const int g_zp = (y + L * zp) * WPR + k, g_zm = (y + L * zm) * WPR + k;
        const uint32_t Sv = *(const uint32_t *)(own + 4 * g);
        const uint32_t Xa = *(const uint32_t *)(oth + 4 * g);
        const uint32_t Xo = *(const uint32_t *)(oth + 4 * g_x);
        const uint32_t Yp = *(const uint32_t *)(oth + 4 * g_yp);
        const uint32_t Ym = *(const uint32_t *)(oth + 4 * g_ym);
        const uint32_t Zp = *(const uint32_t *)(oth + 4 * g_zp);
        const uint32_t Zm = *(const uint32_t *)(oth + 4 * g_zm);
        const uint32_t sel = eps ? 0x00070605u : 0x06050403u;
        const uint32_t Xs = __builtin_amdgcn_perm(Xa, Xo, sel);
        const u32x4 rw = philox4x32_10((uint32_t)g, c1, c2, d.sample_id, A.key0, A.key1);
        uint32_t fm;
        if constexpr (JK == 0) {
            const int *Jp = A.Ju + d.J_off + (size_t)p * 3 * HALF;
            const int *Jo = A.Ju + d.J_off + (size_t)(1 - p) * 3 * HALF;
            const int4 Jpx = *(const int4 *)(Jp + 4 * g);
            const int4 Jpy = *(const int4 *)(Jp + HALF + 4 * g);
            const int4 Jpz = *(const int4 *)(Jp + 2 * HALF + 4 * g);
            const int4 V = *(const int4 *)(Jo + 4 * g);
            const int4 Jym = *(const int4 *)(Jo + HALF + 4 * g_ym);
            const int4 Jzm = *(const int4 *)(Jo + 2 * HALF + 4 * g_zm);
            const int Ep = Jo[row * HL + (k == 0 ? HL - 1 : 4 * k - 1)];
            const int Ja[4] = {eps ? V.x : Jpx.x, eps ? V.y : Jpx.y, eps ? V.z : Jpx.z, eps ? V.w : Jpx.w};
            const int Js[4] = {eps ? Jpx.x : Ep, eps ? Jpx.y : V.x, eps ? Jpx.z : V.y, eps ? Jpx.w : V.z};
            const int Jy[4] = {Jpy.x, Jpy.y, Jpy.z, Jpy.w}, Jyn[4] = {Jym.x, Jym.y, Jym.z, Jym.w};
            const int Jz[4] = {Jpz.x, Jpz.y, Jpz.z, Jpz.w}, Jzn[4] = {Jzm.x, Jzm.y, Jzm.z, Jzm.w};
            const float kav[4] = {ka, ka, ka, ka}, kbv[4] = {kb, kb, kb, kb};
            int Sus[4];
            fm = update_word_gauss<true>(Sv, Xa, Xs, Yp, Ym, Zp, Zm, Ja, Js, Jy, Jyn, Jz, Jzn, rw, kav, kbv,
                                         [=](int) { return 2.0f * b32; }, d.h32, d.hgrid, Sus);
            accE += tally_delta(Sv, fm, Sus);
        } else {
            const uint8_t *J8 = (const uint8_t *)A.J + d.J_off;
            const uint8_t *Jp = J8 + (size_t)p * 3 * HALF, *Jo = J8 + (size_t)(1 - p) * 3 * HALF;
            const uint32_t Jpx = *(const uint32_t *)(Jp + 4 * g);
            const uint32_t Jpy = *(const uint32_t *)(Jp + HALF + 4 * g);
            const uint32_t Jpz = *(const uint32_t *)(Jp + 2 * HALF + 4 * g);
            const uint32_t V = *(const uint32_t *)(Jo + 4 * g);
            const uint32_t Vo = *(const uint32_t *)(Jo + 4 * g_x);
            const uint32_t Jym = *(const uint32_t *)(Jo + HALF + 4 * g_ym);
            const uint32_t Jzm = *(const uint32_t *)(Jo + 2 * HALF + 4 * g_zm);
            const uint32_t Ja = eps ? V : Jpx;
            const uint32_t Js = eps ? Jpx : __builtin_amdgcn_perm(V, Vo, 0x06050403u);
            fm = update_word_pm1(Sv, Xa, Xs, Yp, Ym, Zp, Zm, Ja, Js, Jpy, Jym, Jpz, Jzm, rw, thr, d.down_mask,
                                 accE);
        }
        *(uint32_t *)(own + 4 * g) = Sv ^ fm;
        bf += __builtin_popcount(fm);
        bd += __builtin_popcount(Sv & fm);
    }
    long long sE = accE;
    block_sum3<256>(sE, bf, bd);
    if (tid == 0) {
        const int flips = bf / 7, ndown = bd / 7;
        // sE + ndown = sum over accepted sites of s (S_u + hgrid) (Gaussian), less hgrid sum s
        const long long corr = JK == 0 ? (long long)d.hgrid * (flips - 2 * ndown) : 0;
        atomicAdd((unsigned long long *)&A.dEJ[gi + w], (unsigned long long)(2 * (sE + ndown - corr)));
        atomicAdd(&A.dM[gi + w], -2 * (flips - 2 * ndown));
        atomicAdd((unsigned long long *)&A.flips[gi + t], (unsigned long long)flips);
    }
}

// Exchange pass of one sweep for the HBM tier: one wave per (sample, chain).
__global__ void __launch_bounds__(64) hbm_exchange_kernel(SweepArgs A)
{
    const int code = A.items[blockIdx.x];
    const SampleDev d = A.samples[code >> 1];
    const int r = code & 1;
    const int nT = d.n_T, gi = 2 * d.slot_off + r * nT;
    const int tid = threadIdx.x;
    const int64_t n = A.state[0] + A.it;
    const double unit = A.jkind == 0 ? 0x1p-18 : 1.0;
    const double hd = (double)d.h32;
    if (tid < nT) {
        A.EJ[gi + tid] += A.dEJ[gi + tid];
        A.M[gi + tid] += A.dM[gi + tid];
        A.dEJ[gi + tid] = 0;
        A.dM[gi + tid] = 0;
    }
    __syncthreads();
    for (int j = tid;; j += blockDim.x) {
        const int t = (int)(n & 1) + 2 * j;
        if (t + 1 >= nT) break;
        const int w0 = A.was[gi + t], w1 = A.was[gi + t + 1];
        const double E0 = (double)A.EJ[gi + w0] * unit - hd * (double)A.M[gi + w0];
        const double E1 = (double)A.EJ[gi + w1] * unit - hd * (double)A.M[gi + w1];
        const double D = (A.beta[d.slot_off + t] - A.beta[d.slot_off + t + 1]) * (E0 - E1);
        bool acc = D >= 0.0;
        if (!acc) {
            const u32x4 q = philox4x32_10(0u, (uint32_t)n,
                                          (PURPOSE_EXCHANGE << 28) | ((uint32_t)t << 1) | (uint32_t)r,
                                          d.sample_id, A.key0, A.key1);
            acc = exchange_accept(u53_of(q.x, q.y), D);
        }
        if (acc) {
            A.was[gi + t] = w1;
            A.was[gi + t + 1] = w0;
            A.swaps[gi + t] += 1;
        }
    }
    __syncthreads();
    if (tid < nT) {
        const int w = A.was[gi + tid];
        A.sow[gi + w] = tid;
        const int64_t done = n + 1;
        if (A.measure_every > 0 && done > A.measure_start && (done - A.measure_start) % A.measure_every == 0) {
            const int64_t f = measurements_upto(done, A.measure_every, A.measure_start) -
                              measurements_upto(A.state[0], A.measure_every, A.measure_start) - 1;
            A.frameE[f * 2 * A.total_slots + gi + tid] = (double)A.EJ[gi + w] * unit - hd * (double)A.M[gi + w];
        }
    }
}

// Snapshot of one (sample, chain, slot) for the HBM tier, when a measurement
// is due after this sweep (the launch returns at once otherwise).
__global__ void __launch_bounds__(256) hbm_snapshot_kernel(SweepArgs A)
{
    const int64_t n = A.state[0] + A.it, done = n + 1;
    if (!(A.measure_every > 0 && done > A.measure_start && (done - A.measure_start) % A.measure_every == 0))
        return;
    const int code = A.walkers[blockIdx.x];
    const SampleDev d = A.samples[code >> 7];
    const int r = (code >> 6) & 1, t = code & 63;
    const int L = d.L, L2 = L * L, N = L2 * L, HALF = N / 2;
    const int nT = d.n_T, gi = 2 * d.slot_off + r * nT;
    const int64_t f = measurements_upto(done, A.measure_every, A.measure_start) -
                      measurements_upto(A.state[0], A.measure_every, A.measure_start) - 1;
    const int8_t *Sw = A.spins + d.spin_off + ((size_t)r * nT + A.was[gi + t]) * N;
    uint32_t *dst = A.frames + f * A.frame_words + d.frame_off + ((size_t)r * nT + t) * L2;
    for (int row = threadIdx.x; row < L2; row += blockDim.x) {
        const int yz = (row % L) + row / L;
        uint32_t bits = 0;
        for (int x = 0; x < L; ++x) {
            const int p = (x + yz) & 1;
            bits |= (uint32_t)(Sw[p * HALF + ((x + L * row) >> 1)] < 0) << x;
        }
        dst[row] = bits;
    }
}

#define EA_HBM(Lv)                                                  \
    template __global__ void hbm_half_kernel<Lv, 0, 0>(SweepArgs); \
    template __global__ void hbm_half_kernel<Lv, 1, 0>(SweepArgs); \
    template __global__ void hbm_half_kernel<Lv, 0, 1>(SweepArgs); \
    template __global__ void hbm_half_kernel<Lv, 1, 1>(SweepArgs);
EA_HBM(8)
EA_HBM(16)
EA_HBM(24)
EA_HBM(32)
#undef EA_HBM

// ---------------------------------------------------------------------------
// Overlap measurement (eq. 2).  One wave per (sample, slot).  For each snapshot
// frame of the chunk: the overlap bits e = NOT(a XOR b) of the two chains'
// rows mark q_i = +1; the column counts
//   C[x][y] = #{z : e(x,y,z)},  D[x][z] = #{y : e(x,y,z)},  R[y][z] = #{x : e}
// give the count of q_i = +1 in every plane of the nine wave vectors
// k_f = (2 pi / L) u_f (each plane c = u_f . r mod L holds L^2 sites), so the
// plane sums are P_f[c] = 2 count - L^2 and
// q(k_f) = sum_c P_f[c] e^{2 pi i c / L} / N (summed in c order), added to the
// binary64 accumulators of the slot in time order.
//
// A wave may take F frames side by side, one per group of G = 64 / F lanes,
// each group at least 2 L lanes wide: the frames' counts and Fourier sums are
// independent, and their accumulation stays one frame after the other.
//
// C and D come from bit-sliced vertical counters: lane y of a group (C) adds
// the rows (y, z) over z, lane D0 + z (D) the rows (y, z) over y (D0 = L
// with frames side by side, else 32), one 32-bit word per step into six bit
// planes, and then reads the L column counts off the planes.  Tables in LDS
// use a row stride of L + 1 words, so that the strided reads of the plane
// sums fall in distinct banks.
template <int L, int D0>
__device__ __forceinline__ void column_counts(const uint32_t *eqr, int lane, int *C, int *D)
{
    constexpr int LP = L + 1;
    static_assert(D0 >= L && D0 + L <= 64, "C and D lanes apart");
    const bool isC = lane < L, isD = lane >= D0 && lane < D0 + L;
    if (!isC && !isD) return;
    const int u = isC ? lane : lane - D0;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
#pragma unroll 4
    for (int v = 0; v < L; ++v) {
        const uint32_t w = eqr[isC ? u + LP * v : v + LP * u];
        uint32_t k = c0 & w;
        c0 ^= w;
        uint32_t k2 = c1 & k;
        c1 ^= k;
        k = c2 & k2;
        c2 ^= k2;
        k2 = c3 & k;
        c3 ^= k;
        k = c4 & k2;
        c4 ^= k2;
        c5 |= k;  // counts reach at most L <= 32
    }
    int *dst = isC ? C : D;
#pragma unroll
    for (int x = 0; x < L; ++x) {
        const int cnt = (int)(((c0 >> x) & 1u) | (((c1 >> x) & 1u) << 1) | (((c2 >> x) & 1u) << 2) |
                              (((c3 >> x) & 1u) << 3) | (((c4 >> x) & 1u) << 4) | (((c5 >> x) & 1u) << 5));
        dst[x * LP + u] = cnt;
    }
}

// Frames measured side by side by one wave: as many as groups of 2 L lanes
// fit, at most two (four groups of 16 lanes, at L <= 8, measured no faster
// than one).
template <int L>
constexpr int meas_frames()
{
    return 2 * L <= 32 ? 2 : 1;
}

// LDS of one slot's measurement (per frame group g: the tables of its frame).
template <int L, int F>
struct MeasLds {
    static_assert(F >= 1 && 2 * L * F <= 64, "a group of 2 L lanes per frame");
    static constexpr int LP = L + 1, G = 64 / F;
    static constexpr int GC = G / L;  // chunks of v per plane count
    double accs[NACC];
    double re_f[F][NPLANE], im_f[F][NPLANE];
    double Ea[F], Eb[F];
    double cst[L], snt[L];  // cos and sin of 2 pi c / L
    uint32_t eqr[F][L * LP];
    int C[F][L * LP], D[F][L * LP], R[F][L * LP];
    int P[F][NPLANE][L];
    int part[F][NPLANE][GC][L];
};

// The measurement of slot A.slots[slot_index] by one wave, with its LDS at buf.
template <int L, int F>
__device__ __forceinline__ void measure_slot(const MeasureArgs &A, int slot_index, char *buf)
{
    constexpr int L2 = L * L, LP = L + 1;
    constexpr uint32_t mask = L == 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
    using M = MeasLds<L, F>;
    constexpr int G = M::G, GC = M::GC;
    M &S = *reinterpret_cast<M *>(buf);
    auto &accs = S.accs;
    const int gs = A.slots[slot_index];
    const int s = A.slot_sample[gs];
    const SampleDev d = A.samples[s];
    const int t = gs - d.slot_off;
    const int tid = threadIdx.x, T = blockDim.x;
    const int g = tid / G, lt = tid - g * G;  // frame group, lane within it
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
    for (int c = tid; c < L; c += T) {
        S.cst[c] = A.costab[(size_t)L * MAX_L + c];
        S.snt[c] = A.sintab[(size_t)L * MAX_L + c];
    }
    constexpr double Nd = (double)(L2 * L);
    for (int64_t f0 = 0; f0 < nf; f0 += F) {
        const int64_t f = f0 + g;
        const bool live = f < nf;  // the last batch may hold fewer than F frames
        uint32_t *eqr = S.eqr[g];
        int *C = S.C[g], *D = S.D[g], *R = S.R[g];
        double Ea = 0.0, Eb = 0.0;  // one frame per wave: the accumulating lane's own
        if (live) {
            const uint32_t *ra = A.frames + f * A.frame_words + d.frame_off + (size_t)t * L2;
            const uint32_t *rb = ra + (size_t)d.n_T * L2;
            if (lt == NPLANE) {  // the frame's two energies, loaded early (used by the accumulation)
                const double *E = A.frameE + f * 2 * A.total_slots + 2 * (size_t)d.slot_off;
                Ea = E[t];
                Eb = E[d.n_T + t];
                if constexpr (F > 1) {
                    S.Ea[g] = Ea;
                    S.Eb[g] = Eb;
                }
            }
            for (int i = lt; i < L2; i += G) {
                const uint32_t e = ~(ra[i] ^ rb[i]) & mask;
                const int y = i % L, z = i / L;
                eqr[y + LP * z] = e;
                R[y + LP * z] = __builtin_popcount(e);
            }
        }
        __syncthreads();
        if (live) column_counts<L, F == 1 ? 32 : L>(eqr, lt, C, D);  // C[x][y] at x*LP + y, D[x][z] at x*LP + z
        __syncthreads();
        // plane counts: lane (c, chunk) sums v = chunk, chunk + GC, ... of
        // every family (no divergence: the family loop is unrolled), then
        // (family, c) tasks add the GC chunk partials (integers: any order)
        if (live && lt < L * GC) {
            const int c = lt % L, chunk = lt / L;
#pragma unroll
            for (int fam = 0; fam < NPLANE; ++fam) {
                int cnt = 0;
                for (int v = chunk; v < L; v += GC) {
                    const int cm = c - v < 0 ? c - v + L : c - v;    // c - v mod L
                    const int cp = c + v >= L ? c + v - L : c + v;   // c + v mod L
                    const int vm = v - c < 0 ? v - c + L : v - c;    // v - c mod L
                    if (fam == 0) cnt += C[c * LP + v];        // x = c
                    else if (fam == 1) cnt += C[v * LP + c];   // y = c
                    else if (fam == 2) cnt += D[v * LP + c];   // z = c
                    else if (fam == 3) cnt += C[cm * LP + v];  // x + y = c
                    else if (fam == 4) cnt += C[cp * LP + v];  // x - y = c
                    else if (fam == 5) cnt += D[cm * LP + v];  // x + z = c
                    else if (fam == 6) cnt += D[cp * LP + v];  // x - z = c
                    else if (fam == 7) cnt += R[v + LP * cm];  // y + z = c
                    else cnt += R[v + LP * vm];                // y - z = c
                }
                S.part[g][fam][chunk][c] = cnt;
            }
        }
        __syncthreads();
        if (live) {
            for (int task = lt; task < NPLANE * L; task += G) {
                const int fam = task / L, c = task - fam * L;
                int cnt = 0;
                for (int k = 0; k < GC; ++k) cnt += S.part[g][fam][k][c];
                S.P[g][fam][c] = 2 * cnt - L2;
            }
        }
        __syncthreads();
        if (live && lt < NPLANE) {
            double re = 0.0, im = 0.0;
            for (int c = 0; c < L; ++c) {
                re += (double)S.P[g][lt][c] * S.cst[c];
                im += (double)S.P[g][lt][c] * S.snt[c];
            }
            S.re_f[g][lt] = re / Nd;
            S.im_f[g][lt] = im / Nd;
        }
        __syncthreads();
        // the batch's frames into the accumulators, in time order
        const int nb = F == 1 ? 1 : nf - f0 < F ? (int)(nf - f0) : F;
        if (tid < NPLANE) {
            for (int k = 0; k < nb; ++k) {
                const double re = S.re_f[k][tid], im = S.im_f[k][tid];
                accs[5 + 3 * tid] += re;
                accs[6 + 3 * tid] += im;
                accs[7 + 3 * tid] += re * re + im * im;
            }
        } else if (tid == NPLANE) {
            for (int k = 0; k < nb; ++k) {
                int S0 = 0;
                for (int c = 0; c < L; ++c) S0 += S.P[k][0][c];
                const double q0 = (double)S0 / Nd;
                accs[0] += 1.0;
                accs[1] += q0;
                accs[2] += q0 * q0;
                accs[3] += (q0 * q0) * q0;
                accs[4] += (q0 * q0) * (q0 * q0);
                const double ea = F == 1 ? Ea : S.Ea[k], eb = F == 1 ? Eb : S.Eb[k];
                accs[32] += ea;
                accs[33] += ea * ea;
                accs[34] += eb;
                accs[35] += eb * eb;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < NACC; i += T) A.acc[(size_t)gs * NACC + i] = accs[i];
}

template <int L>
__global__ void __launch_bounds__(64) measure_kernel(MeasureArgs A)
{
    __shared__ __attribute__((aligned(16))) char buf[sizeof(MeasLds<L, meas_frames<L>()>)];
    measure_slot<L, meas_frames<L>()>(A, blockIdx.x, buf);
}

#define EA_MEAS(Lv) template __global__ void measure_kernel<Lv>(MeasureArgs);
EA_MEAS(2)
EA_MEAS(4)
EA_MEAS(6)
EA_MEAS(8)
EA_MEAS(10)
EA_MEAS(12)
EA_MEAS(14)
EA_MEAS(16)
EA_MEAS(24)
EA_MEAS(32)
#undef EA_MEAS

// Neighbouring binary32 values (by bit pattern; -0 and +0 step to the
// smallest subnormals, infinities stay).
__device__ __forceinline__ float float_up(float v)
{
    if (v == __builtin_inff()) return v;
    if (v == 0.0f) return __uint_as_float(1u);
    const uint32_t b = __float_as_uint(v);
    return __uint_as_float(v > 0.0f ? b + 1u : b - 1u);
}
__device__ __forceinline__ float float_down(float v) { return -float_up(-v); }

// Exhaustive check of the acceptance gap used by the row, group and HBM
// engines, in binary64, with M = ACCEPT_MARGIN.  One thread per binary32 bit
// pattern v (NaNs excluded by the launch):
// (1) the hardware exponential is monotone: 2^v <= 2^(next binary32 above v);
// (2) for x = v: every exponent y the engines can form for x lies within a
//     relative 2^-21 of z = x log2(e) plus an absolute 2^-20 (the roundings of
//     both forms in update_word_gauss: at most about 5 2^-24 relative, plus
//     2 beta32 log2(e) 2^-19 2^-24 < 2^-20 from the field remainder's constant
//     of the folded form for beta32 <= 2^20); with yl, yh the binary32 values just
//     outside that interval and A = 2^y 2^32 at both ends (exact here),
//     T = exp_ea32(x) 2^32 (0 below -86):
//       x <= 0:  T - (M - 384) <= A(yl)  and  A(yh) <= T + (M - 128)
//       x > 0:   A(yl) >= 2^32 - M + 384   (dE < 0: the exact test accepts)
// Also records the largest |A / T - 1| at the two ends over [-86, 0].
__global__ void exp_bracket_kernel(uint32_t first_bits, uint32_t count, unsigned long long *violations,
                                   unsigned int *max_dev_bits)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = __uint_as_float(first_bits + i);
    bool ok = true;
    if (v != __builtin_inff() && !(__builtin_amdgcn_exp2f(v) <= __builtin_amdgcn_exp2f(float_up(v)))) ok = false;

    const double TWO32 = 4294967296.0, M = ACCEPT_MARGIN;
    const double z = (double)v * (double)__uint_as_float(0x3FB8AA3Bu);  // exact: 24 x 24 bits
    const double B = 0x1p-21, D = 0x1p-20;
    const double zl = (z <= 0.0 ? z * (1.0 + B) : z * (1.0 - B)) - D;
    const double zh = (z <= 0.0 ? z * (1.0 - B) : z * (1.0 + B)) + D;
    float yl = (float)zl, yh = (float)zh;
    if ((double)yl > zl) yl = float_down(yl);
    if ((double)yh < zh) yh = float_up(yh);
    const double Al = (double)__builtin_amdgcn_exp2f(yl) * TWO32;
    const double Ah = (double)__builtin_amdgcn_exp2f(yh) * TWO32;
    if (v > 0.0f) {
        ok = ok && Al >= TWO32 - M + 384.0;
    } else {
        const double T = v >= -86.0f ? (double)exp_ea32(v) * TWO32 : 0.0;
        ok = ok && Al >= T - (M - 384.0) && Ah <= T + (M - 128.0);
        if (v >= -86.0f) {
            const float dev = (float)(fmax(fabs(Al - T), fabs(Ah - T)) / T);
            atomicMax(max_dev_bits, __float_as_uint(dev));
        }
    }
    if (!ok) atomicAdd(violations, 1ull);
}

// The replica-exchange shortcut (exchange_accept in ea_device.hpp), one
// thread per binary32 bit pattern y from -0 down to -58: the hardware
// exponential lies within a relative 2^-22 of 2^y (binary64 exp2 as the
// reference) and exp_ea64(y) within 2^-49 of e^y (binary64 exp, itself within
// an ulp); records the largest |2^y (hardware) / 2^y - 1|.  With D = 1.5 y
// (down to -87, past the cut at -40) it also compares the decision itself
// with u < exp_ea64(D) for uniforms on the 2^-53 grid at relative distances
// k 2^-17 (k = -6 .. 6) from exp_ea64(D), both sides of the margin, and for
// u = 0 and u = 1 - 2^-53.
__global__ void exchange_bracket_kernel(uint32_t first_bits, uint32_t count, unsigned long long *violations,
                                        unsigned long long *max_dev_bits)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float y = __uint_as_float(first_bits + i);
    const double dev = fabs((double)__builtin_amdgcn_exp2f(y) / exp2((double)y) - 1.0);
    bool ok = dev <= 0x1p-22 && fabs(exp_ea64((double)y) / exp((double)y) - 1.0) <= 0x1p-49;
    if (y < 0.0f) {
        const double D = 1.5 * (double)y, E = exp_ea64(D);
        ok = ok && exchange_accept(0.0, D) == (0.0 < E) && exchange_accept(1.0 - 0x1p-53, D) == (1.0 - 0x1p-53 < E);
        for (int k = -6; k <= 6; ++k) {
            const double u = fmin(floor(E * (1.0 + k * 0x1p-17) * 0x1p53) * 0x1p-53, 1.0 - 0x1p-53);
            ok = ok && exchange_accept(u, D) == (u < E);
        }
    }
    atomicMax(max_dev_bits, (unsigned long long)__double_as_longlong(dev));
    if (!ok) atomicAdd(violations, 1ull);
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

// Snapshot of the current state (slot order, bit rows) into frame 0, for an
// immediate measurement.  One workgroup per (sample, chain).
__global__ void __launch_bounds__(256) snapshot_kernel(const SampleDev *samples, const int32_t *items,
                                                      const int8_t *spins, const int32_t *was,
                                                      const int64_t *EJ, const int32_t *M, int jkind,
                                                      uint32_t *frame, double *frameE)
{
    const int code = items[blockIdx.x];
    const SampleDev d = samples[code >> 1];
    const int r = code & 1;
    const int L = d.L, L2 = L * L, N = L2 * L, HALF = N / 2;
    const size_t sbase = (size_t)d.spin_off + (size_t)r * d.n_T * N;
    const int gi = 2 * d.slot_off + r * d.n_T;
    uint32_t *dst = frame + d.frame_off + (size_t)r * d.n_T * L2;
    for (int i = threadIdx.x; i < d.n_T * L2; i += blockDim.x) {
        const int t = i / L2, row = i - t * L2;
        const int8_t *Sw = spins + sbase + (size_t)was[gi + t] * N;
        const int yz = (row % L) + row / L;
        uint32_t bits = 0;
        for (int x = 0; x < L; ++x) {
            const int p = (x + yz) & 1;
            bits |= (uint32_t)(Sw[p * HALF + ((x + L * row) >> 1)] < 0) << x;
        }
        dst[i] = bits;
    }
    const double unit = jkind == 0 ? 0x1p-18 : 1.0;
    for (int t = threadIdx.x; t < d.n_T; t += blockDim.x) {
        const int w = was[gi + t];
        frameE[gi + t] = (double)EJ[gi + w] * unit - (double)d.h32 * (double)M[gi + w];
    }
}

}  // namespace ea
