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
// measurement, the finalize and the setup and check kernels.
#include "ea_device.hpp"
#include "ea_exact.hpp"
#include "ea_item.hpp"
#include "ea_types.hpp"
#include "ea_update.hpp"

namespace ea {

// ---------------------------------------------------------------------------
// Site engine: one checkerboard half-sweep (parity p) over every walker of the
// chain.  A thread takes groups of four consecutive sublattice sites (one
// Philox call, word h&3 for site h) of one walker; sites of one parity never
// neighbour each other, so the updates of a half-sweep are independent.
template <int L, int JK>
__device__ __forceinline__ void site_half_sweep(const SweepArgs &A, const SampleDev &d, int r, int p,
                                                int64_t n, const ItemLds &I)
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
            t = I.sow[w];
            const u32x4 rw = philox4x32_10((uint32_t)g, c1, c2base | ((uint32_t)t << 1), d.sample_id,
                                           A.key0, A.key1);
            const uint32_t words[4] = {rw.x, rw.y, rw.z, rw.w};
            int8_t *Sp = I.S + (size_t)w * item_walker_stride(L) + p * HALF;
            const int8_t *So = I.S + (size_t)w * item_walker_stride(L) + (1 - p) * HALF;
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
                    const float *Jp = (const float *)I.J + p * 3 * HALF;
                    const float *Jo = (const float *)I.J + (1 - p) * 3 * HALF;
                    // exact: every partial sum is a multiple of 2^-18 below 2^6
                    float SJ = Jp[h] * (float)s0;
                    SJ = SJ + Jo[hxm] * (float)s1;
                    SJ = SJ + Jp[HALF + h] * (float)s2;
                    SJ = SJ + Jo[HALF + hym] * (float)s3;
                    SJ = SJ + Jp[2 * HALF + h] * (float)s4;
                    SJ = SJ + Jo[2 * HALF + hzm] * (float)s5;
                    const float f = SJ + d.h32;
                    const float dE = (2.0f * (float)si) * f;
                    const float e = exp_ea32(-(I.b32[t] * dE));
                    accept = (dE <= 0.0f) | (u24_of(words[i]) < e);
                    units = (int)(SJ * 262144.0f);
                } else {
                    const int8_t *Jp = (const int8_t *)I.J + p * 3 * HALF;
                    const int8_t *Jo = (const int8_t *)I.J + (1 - p) * 3 * HALF;
                    const int SJ = Jp[h] * s0 + Jo[hxm] * s1 + Jp[HALF + h] * s2 +
                                   Jo[HALF + hym] * s3 + Jp[2 * HALF + h] * s4 +
                                   Jo[2 * HALF + hzm] * s5;
                    const float f = (float)SJ + d.h32;  // sign of SJ + h is exact
                    const bool down = si * f <= 0.0f;
                    const uint32_t thr = I.lut[(t * 2 + ((si + 1) >> 1)) * 7 + ((SJ + 6) >> 1)];
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
                    atomicAdd((unsigned long long *)&I.dEJ[w0], (unsigned long long)se);
                    atomicAdd(&I.dM[w0], (pk - sfl) / 65536);
                    atomicAdd(&I.fl[I.sow[w0]], sfl);
                }
            }
        } else if (act) {
            atomicAdd((unsigned long long *)&I.dEJ[w], (unsigned long long)(long long)dEu);
            atomicAdd(&I.dM[w], dm);
            atomicAdd(&I.fl[t], nfl);
        }
    }
}

// The same for +-1 couplings (int8x4 bond words Ja..Jzn): a bond-spin product
// byte n ^ J is 0x00 for +1 and 0xFE for -1, so per byte c = number of -1
// products and S_J = 6 - 2c.  Acceptance uses the slot's threshold table
// thr[a*7 + b] (a = (s_i+1)/2, b = (S_J+6)/2): accept iff dE <= 0 (bit a*7+b of
// down_mask, set on the host from 2 s (S_J + h) <= 0) or w < thr.  S_u = S_J.
__device__ __forceinline__ uint32_t update_word_pm1(uint32_t Sv, uint32_t Xa, uint32_t Xs, uint32_t Yp, uint32_t Ym,
                                                    uint32_t Zp, uint32_t Zm, uint32_t Ja, uint32_t Js, uint32_t Jy,
                                                    uint32_t Jyn, uint32_t Jz, uint32_t Jzn, const u32x4 rw,
                                                    const uint32_t *thr, uint32_t down_mask, int &accE)
{
    constexpr uint32_t LOW = 0x01010101u;
    const uint32_t cnt = (((Xa ^ Ja) >> 1) & LOW) + (((Xs ^ Js) >> 1) & LOW) + (((Yp ^ Jy) >> 1) & LOW) +
                         (((Ym ^ Jyn) >> 1) & LOW) + (((Zp ^ Jz) >> 1) & LOW) + (((Zm ^ Jzn) >> 1) & LOW);
    const uint32_t words[4] = {rw.x, rw.y, rw.z, rw.w};
    uint32_t fm = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int sh = 8 * i;
        const int b = 6 - (int)((cnt >> sh) & 0xFFu);               // (S_J + 6) / 2
        const int m = __builtin_amdgcn_sbfe((int)Sv, sh + 7, 1);  // 0: s_i = +1, -1: s_i = -1
        const int idx = (m + 1) * 7 + b;
        const bool accept = ((down_mask >> idx) & 1u) | (words[i] < thr[idx]);
        if (accept) {
            fm |= 0xFEu << sh;
            accE += (2 * b - 6) ^ m;
        }
    }
    return fm;
}

// ---------------------------------------------------------------------------
// Row engine (L = 8 or 16, Gaussian couplings held as int32 multiples of
// 2^-18).  Sublattice p's row (y, z) holds L/2 sites, i.e. L/8 int8x4 words;
// site h = 4g + i of the row's word g sits at x = 2(4k + i) + eps with
// eps = (y + z + p) & 1.  Its x-neighbours in the other sublattice are the
// sites of the same word index ("aligned", x + 1 if eps = 0, else x - 1) and
// the sites one position over ("shifted": x - 1 if eps = 0, else x + 1), which
// one byte permute of the row's words produces.  The y and z neighbours are
// the words of the same index in the adjacent rows.
//
// Tallies per thread and sweep: the first half-sweep tallies no energy; the
// second gives accE + nd = sum of s_i S_u over the thread's odd sites after
// the update (tally_final), i.e. minus its share of the walker's new E_J;
// bf and bd count the set bits of the flip masks (7 per flipped byte) and of
// (spins AND flip mask) over both halves.
//
// Lane map: a walker's L*L/8 columns (k, y) are split by the parity of y over
// two waves, and a wave holds the columns of WPW walkers with y of one parity.
// eps = (y + z + p) & 1 is then the same for every lane of a wave, so each
// parity of z has its own specialised code path with no per-lane selects.
template <int L>
struct RowMap {
    static constexpr int WPR = L / 8, HL = L / 2;
    static constexpr int CPW = WPR * HL;  // columns of one y-parity per walker
    static constexpr int WPW = 64 / CPW;  // walkers per wave
};

// Row engine coupling layout in LDS: within each z plane the rows y are stored
// in the order of row_slot (even y, then odd y), so the columns a wave holds
// (one y parity) read one contiguous run of 16-byte coupling words.
template <int L>
__device__ __forceinline__ int row_slot(int y)
{
    return (y & 1) * (L / 2) + (y >> 1);
}

// j_y0, j_ym, je_prev: the coupling offsets of the word and of its -y neighbour
// word, and the coupling element before the word, in that layout.
template <int L, int P, int EPS>
__device__ __forceinline__ void row_word(const SweepArgs &A, const SampleDev &d, uint8_t *Sw, const int *J,
                                         int o_y0, int o_yp, int o_ym, int o_x, int j_y0, int j_ym, int je_prev,
                                         int z, int zp, int zm, uint32_t c1, uint32_t c2, float ka, float kb,
                                         float h32, int &accE, int &nd, int &bf, int &bd)
{
    constexpr int HALF = L * L * L / 2, HL = L / 2, PLANE = L * HL;
    const uint8_t *own = Sw + P * HALF, *oth = Sw + (1 - P) * HALF;
    const int *Jp = J + P * 3 * HALF, *Jo = J + (1 - P) * 3 * HALF;
    const int zo = z * PLANE;
    const uint32_t Sv = *(const uint32_t *)(own + o_y0 + zo);
    const uint32_t Xa = *(const uint32_t *)(oth + o_y0 + zo);
    const uint32_t Xo = L == 8 ? Xa : *(const uint32_t *)(oth + o_x + zo);
    const uint32_t Yp = *(const uint32_t *)(oth + o_yp + zo);
    const uint32_t Ym = *(const uint32_t *)(oth + o_ym + zo);
    const uint32_t Zp = *(const uint32_t *)(oth + o_y0 + zp * PLANE);
    const uint32_t Zm = *(const uint32_t *)(oth + o_y0 + zm * PLANE);
    const uint32_t Xs = __builtin_amdgcn_perm(Xa, Xo, EPS ? 0x00070605u : 0x06050403u);
    const int4 Jpx = *(const int4 *)(Jp + j_y0 + zo);
    const int4 Jpy = *(const int4 *)(Jp + HALF + j_y0 + zo);
    const int4 Jpz = *(const int4 *)(Jp + 2 * HALF + j_y0 + zo);
    const int4 V = *(const int4 *)(Jo + j_y0 + zo);
    const int4 Jym = *(const int4 *)(Jo + HALF + j_ym + zo);
    const int4 Jzm = *(const int4 *)(Jo + 2 * HALF + j_y0 + zm * PLANE);
    // bonds to the aligned x-neighbour (x+1 if eps = 0, else x-1) and the shifted one
    int Ja[4], Js[4];
    if constexpr (EPS) {
        Ja[0] = V.x; Ja[1] = V.y; Ja[2] = V.z; Ja[3] = V.w;
        Js[0] = Jpx.x; Js[1] = Jpx.y; Js[2] = Jpx.z; Js[3] = Jpx.w;
    } else {
        const int Ep = Jo[je_prev + zo];
        Ja[0] = Jpx.x; Ja[1] = Jpx.y; Ja[2] = Jpx.z; Ja[3] = Jpx.w;
        Js[0] = Ep; Js[1] = V.x; Js[2] = V.y; Js[3] = V.z;
    }
    const int Jy[4] = {Jpy.x, Jpy.y, Jpy.z, Jpy.w}, Jyn[4] = {Jym.x, Jym.y, Jym.z, Jym.w};
    const int Jz[4] = {Jpz.x, Jpz.y, Jpz.z, Jpz.w}, Jzn[4] = {Jzm.x, Jzm.y, Jzm.z, Jzm.w};
    const uint32_t g = (uint32_t)(o_y0 / 4 + z * (PLANE / 4));
    const u32x4 rw = philox4x32_10(g, c1, c2, d.sample_id, A.key0, A.key1);
    const float kav[4] = {ka, ka, ka, ka}, kbv[4] = {kb, kb, kb, kb};
    int Sus[4];
    const uint32_t fm = update_word_gauss<true>(
        Sv, Xa, Xs, Yp, Ym, Zp, Zm, Ja, Js, Jy, Jyn, Jz, Jzn, rw, kav, kbv,
        [&](int) { return 2.0f * A.beta32[d.slot_off + ((c2 >> 1) & 0x7FFFFFFu)]; }, h32, d.hgrid, Sus);
    if constexpr (P == 1) tally_final(Sv, fm, Sus, accE, nd);
    *(uint32_t *)(Sw + P * HALF + o_y0 + zo) = Sv ^ fm;
    bf += __builtin_popcount(fm);
    bd += __builtin_popcount(Sv & fm);
}

// Half-sweep P of one walker's column (k, y); E0 = eps of the even z planes.
template <int L, int P, int E0>
__device__ __forceinline__ void row_half_sweep(const SweepArgs &A, const SampleDev &d, int r, int64_t n,
                                               const ItemLds &I, int w, int y, int k, int t, int &accE,
                                               int &nd, int &bf, int &bd)
{
    constexpr int WPR = L / 8, HL = L / 2;
    const int yp = (y + 1) & (L - 1), ym = (y - 1) & (L - 1);
    const int kx = WPR == 2 ? (k ^ 1) : k;
    const int o_y0 = 4 * (y * WPR + k), o_yp = 4 * (yp * WPR + k), o_ym = 4 * (ym * WPR + k);
    const int o_x = 4 * (y * WPR + kx);
    const int j_y0 = 4 * (row_slot<L>(y) * WPR + k), j_ym = 4 * (row_slot<L>(ym) * WPR + k);
    const int je_prev = row_slot<L>(y) * HL + (k == 0 ? HL - 1 : 4 * k - 1);  // element before the word, cyclic
    uint8_t *Sw = (uint8_t *)I.S + (size_t)w * item_walker_stride(L);
    const int *J = (const int *)I.J;
    const uint32_t c1 = (uint32_t)(2 * n + P);
    const uint32_t c2 = (PURPOSE_METROPOLIS << 28) | ((uint32_t)t << 1) | (uint32_t)r;
    // the exponent's two per-slot constants (see update_word_gauss)
    const float cp = two_beta_log2e(I.b32[t]);
    const float ka = cp * 0x1p-18f, kb = cp * (d.h32 - (float)d.hgrid * 0x1p-18f);
    float h32 = d.h32;  // exact path only
#pragma unroll 1
    for (int z = 0; z < L; z += 4) {
        const int zm = z == 0 ? L - 1 : z - 1, z4 = z + 4 == L ? 0 : z + 4;
        row_word<L, P, E0>(A, d, Sw, J, o_y0, o_yp, o_ym, o_x, j_y0, j_ym, je_prev, z, z + 1, zm, c1, c2, ka, kb,
                           h32, accE, nd, bf, bd);
        row_word<L, P, 1 - E0>(A, d, Sw, J, o_y0, o_yp, o_ym, o_x, j_y0, j_ym, je_prev, z + 1, z + 2, z, c1, c2,
                               ka, kb, h32, accE, nd, bf, bd);
        row_word<L, P, E0>(A, d, Sw, J, o_y0, o_yp, o_ym, o_x, j_y0, j_ym, je_prev, z + 2, z + 3, z + 1, c1, c2,
                           ka, kb, h32, accE, nd, bf, bd);
        row_word<L, P, 1 - E0>(A, d, Sw, J, o_y0, o_yp, o_ym, o_x, j_y0, j_ym, je_prev, z + 3, z4, z + 2, c1, c2,
                               ka, kb, h32, accE, nd, bf, bd);
    }
}

// One snapshot row: bit x set iff the spin at (x, y, z) is -1, for the row
// index row = y + L z of a walker held in LDS in sublattice layout.
template <int L>
__device__ __forceinline__ uint32_t pack_row_lds(const int8_t *Sw, int row)
{
    constexpr int HALF = L * L * L / 2, HL = L / 2;
    const int yz = (row % L) + row / L;
    uint32_t bits = 0;
    if constexpr (L % 8 == 0) {
        // The row's HL bytes in each half are its sites in x order, the even x
        // in half (yz & 1), the odd x in the other.  Per 8 sites: two byte
        // permutes interleave them (x = 8g .. 8g+3 and 8g+4 .. 8g+7), the sign
        // bits go to bits 3 and 7 of each byte, and one multiply by
        // 2^21 + 2^14 + 2^7 + 1 carries the sign of x = 8g + k to bit 24 + k
        // (the other partial products fall on distinct bits below 24 or
        // beyond 31, so nothing carries into the result).
        const uint32_t *h0 = (const uint32_t *)(Sw + row * HL), *h1 = (const uint32_t *)(Sw + HALF + row * HL);
        const uint32_t flip = (yz & 1) ? 0x04040404u : 0u;
        const uint32_t sel_lo = 0x05010400u ^ flip, sel_hi = 0x07030602u ^ flip;
#pragma unroll
        for (int g = 0; g < L / 8; ++g) {
            const uint32_t a = h0[g], b = h1[g];
            const uint32_t lo = __builtin_amdgcn_perm(b, a, sel_lo), hi = __builtin_amdgcn_perm(b, a, sel_hi);
            const uint32_t m = ((lo & 0x80808080u) >> 4) | (hi & 0x80808080u);
            bits |= ((m * 0x00204081u) >> 24) << (8 * g);
        }
    } else {
#pragma unroll
        for (int x = 0; x < L; ++x) {
            const int p = (x + yz) & 1;
            bits |= (uint32_t)(Sw[p * HALF + ((x + L * row) >> 1)] < 0) << x;
        }
    }
    return bits;
}

// ---------------------------------------------------------------------------
// The per-item frame shared by both engines.
template <int L, int JK, bool ROW>
__device__ __forceinline__ void run_item(const SweepArgs &A, const SampleDev &d, int r, char *smem)
{
    constexpr int N = L * L * L;
    const int nT = d.n_T;
    const int T = blockDim.x, tid = threadIdx.x;
    const ItemLds I = item_lds(smem, L, nT, JK);

    const size_t sbase = (size_t)d.spin_off + (size_t)r * nT * N;
    const int gi = 2 * d.slot_off + r * nT;
    copy_walkers(I.S, item_walker_stride(L), A.spins + sbase, nT, N, true);
    if constexpr (ROW) {
        // couplings as exact int32 multiples of 2^-18, rows of each z plane
        // placed by row_slot (4 consecutive elements stay within one row)
        constexpr int HALF = N / 2, HL = L / 2, PLANE = L * HL;
        const float4 *src = (const float4 *)((const float *)A.J + d.J_off);  // J_off is a multiple of 4
        int4 *dst = (int4 *)I.J;
        for (int i = tid; i < 3 * N / 4; i += T) {
            const float4 v = src[i];
            const int e = 4 * i, pd = e / HALF, h = e - pd * HALF;
            const int row = h / HL, j = h - row * HL, y = row % L, z = row / L;
            dst[(pd * HALF + z * PLANE + row_slot<L>(y) * HL + j) / 4] =
                make_int4((int)(v.x * 262144.0f), (int)(v.y * 262144.0f), (int)(v.z * 262144.0f),
                          (int)(v.w * 262144.0f));
        }
    } else {
        block_copy(I.J, (const char *)A.J + (size_t)d.J_off * (JK == 0 ? 4 : 1),
                   (size_t)3 * N * (JK == 0 ? 4 : 1));
    }
    for (int i = tid; i < nT; i += T) {
        I.was[i] = A.was[gi + i];
        I.sow[A.was[gi + i]] = i;  // kept by exchange_pass from here on
        I.dEJ[i] = 0;
        I.dM[i] = 0;
        I.EJ[i] = A.EJ[gi + i];
        I.M[i] = A.M[gi + i];
        I.fl[i] = 0;
        I.sw[i] = 0;
        I.b32[i] = A.beta32[d.slot_off + i];
        I.b64[i] = A.beta[d.slot_off + i];
    }
    if (JK == 1)
        for (int i = tid; i < nT * 14; i += T) I.lut[i] = A.lut[(size_t)d.slot_off * 14 + i];
    __syncthreads();

    // row engine: this thread's walker and column (see RowMap)
    constexpr int CPW = RowMap<(L >= 8 ? L : 8)>::CPW, WPW = RowMap<(L >= 8 ? L : 8)>::WPW;
    constexpr int WPR = L / 8 > 0 ? L / 8 : 1;
    const int rw_wave = tid >> 6, rw_lane = tid & 63;
    const int rw_par = __builtin_amdgcn_readfirstlane(rw_wave & 1);
    const int rw_rem = rw_lane % CPW;
    const int rw_w = (rw_wave >> 1) * WPW + rw_lane / CPW;
    const int rw_k = rw_rem % WPR, rw_y = 2 * (rw_rem / WPR) + rw_par;

    const double unit = JK == 0 ? 0x1p-18 : 1.0;
    const double hd = (double)d.h32;
    const int64_t n0 = A.state[0];
    int64_t next_meas = next_measurement(n0, A.measure_every, A.measure_start);
    int64_t f = 0;  // frame of the next measurement within this chunk
    for (int it = 0; it < A.K; ++it) {
        const int64_t n = n0 + it;
        if constexpr (ROW) {
            // Barriers stay outside the walker test: a wave may hold lanes of
            // an active and an idle walker.  A walker's CPW lanes in a wave are
            // aligned and all active or all idle, so the group sums see only
            // its lanes; the two waves of a walker add into LDS.
            const bool on = rw_w < nT;
            const int t = on ? I.sow[rw_w] : 0;
            int accE = 0, nd = 0, bf = 0, bd = 0;
            if (on) {
                if (rw_par) row_half_sweep<L, 0, 1>(A, d, r, n, I, rw_w, rw_y, rw_k, t, accE, nd, bf, bd);
                else row_half_sweep<L, 0, 0>(A, d, r, n, I, rw_w, rw_y, rw_k, t, accE, nd, bf, bd);
            }
            __syncthreads();
            if (on) {
                if (rw_par) row_half_sweep<L, 1, 0>(A, d, r, n, I, rw_w, rw_y, rw_k, t, accE, nd, bf, bd);
                else row_half_sweep<L, 1, 1>(A, d, r, n, I, rw_w, rw_y, rw_k, t, accE, nd, bf, bd);
                // accE + nd = sum of s' (S_u + hgrid) over this thread's 4 L odd
                // sites, |accE| <= 64 sites x 12 2^21 < 2^31; less hgrid sum s'
                const long long sE =
                    group_sum_i64<CPW>((long long)accE + nd - (long long)d.hgrid * (4 * L - 2 * nd));
                const int sf = group_sum_i32<CPW>(bf), sd = group_sum_i32<CPW>(bd);
                if (rw_rem == 0) {
                    const int flips = sf / 7, ndown = sd / 7;
                    // dEJ collects minus the new E_J (both waves of the walker add)
                    atomicAdd((unsigned long long *)&I.dEJ[rw_w], (unsigned long long)sE);
                    atomicAdd(&I.dM[rw_w], -2 * (flips - 2 * ndown));
                    atomicAdd(&I.fl[t], flips);
                }
            }
        } else {
            site_half_sweep<L, JK>(A, d, r, 0, n, I);
            __syncthreads();
            site_half_sweep<L, JK>(A, d, r, 1, n, I);
        }
        __syncthreads();
        for (int i = tid; i < nT; i += T) {
            I.EJ[i] = ROW ? -I.dEJ[i] : I.EJ[i] + I.dEJ[i];
            I.M[i] += I.dM[i];
            I.dEJ[i] = 0;  // cleared for the next sweep's tallies
            I.dM[i] = 0;
        }
        __syncthreads();
        exchange_pass(A, d, r, n, I, unit, hd);
        __syncthreads();
        // Snapshot for the overlap measurement, in slot order.
        const int64_t done = n + 1;
        if (done == next_meas) {
            next_meas += A.measure_every;
            uint32_t *dst = A.frames + f * A.frame_words + d.frame_off + (size_t)r * nT * L * L;
            for (int i = tid; i < nT * L * L; i += T) {
                const int t = i / (L * L), row = i - t * (L * L);
                dst[i] = pack_row_lds<L>(I.S + (size_t)I.was[t] * item_walker_stride(L), row);
            }
            for (int t = tid; t < nT; t += T) {
                const int w = I.was[t];
                A.frameE[f * 2 * A.total_slots + gi + t] = (double)I.EJ[w] * unit - hd * (double)I.M[w];
            }
            ++f;
            __syncthreads();  // the next sweep changes the spins read here
        }
    }
    __syncthreads();
    copy_walkers(I.S, item_walker_stride(L), A.spins + sbase, nT, N, false);
    for (int i = tid; i < nT; i += T) {
        A.was[gi + i] = I.was[i];
        A.EJ[gi + i] = I.EJ[i];
        A.M[gi + i] = I.M[i];
        A.flips[gi + i] += I.fl[i];
        A.swaps[gi + i] += I.sw[i];
    }
    __syncthreads();
}

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
            acc = u53_of(q.x, q.y) < exp_ea64(D);
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
// frame of the chunk, in time order: the overlap bits e = NOT(a XOR b) of the
// two chains' rows mark q_i = +1; the column counts
//   C[x][y] = #{z : e(x,y,z)},  D[x][z] = #{y : e(x,y,z)},  R[y][z] = #{x : e}
// give the count of q_i = +1 in every plane of the nine wave vectors
// k_f = (2 pi / L) u_f (each plane c = u_f . r mod L holds L^2 sites), so the
// plane sums are P_f[c] = 2 count - L^2 and
// q(k_f) = sum_c P_f[c] e^{2 pi i c / L} / N (summed in c order), added to the
// binary64 accumulators of the slot in time order.
//
// C and D come from bit-sliced vertical counters: lane y (C) adds the rows
// (y, z) over z, lane 32 + z (D) the rows (y, z) over y, one 32-bit word per
// step into six bit planes, and then reads the L column counts off the
// planes.  Tables in LDS use a row stride of L + 1 words, so that the strided
// reads of the plane sums fall in distinct banks.
template <int L>
__device__ __forceinline__ void column_counts(const uint32_t *eqr, int lane, int *C, int *D)
{
    constexpr int LP = L + 1;
    const bool isC = lane < L, isD = lane >= 32 && lane - 32 < L;
    if (!isC && !isD) return;
    const int u = isC ? lane : lane - 32;
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

template <int L>
__global__ void __launch_bounds__(64) measure_kernel(MeasureArgs A)
{
    constexpr int L2 = L * L, LP = L + 1;
    constexpr uint32_t mask = L == 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
    __shared__ uint32_t eqr[L * LP];
    __shared__ int C[L * LP], D[L * LP], R[L * LP];
    constexpr int GC = 64 / L;  // chunks of v per plane count
    __shared__ int P[NPLANE][L];
    __shared__ int part[NPLANE][GC][L];
    __shared__ double accs[NACC];
    __shared__ double re_f[NPLANE], im_f[NPLANE];
    __shared__ double cst[L], snt[L];  // cos and sin of 2 pi c / L
    const int gs = A.slots[blockIdx.x];
    const int s = A.slot_sample[gs];
    const SampleDev d = A.samples[s];
    const int t = gs - d.slot_off;
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
    for (int c = tid; c < L; c += T) {
        cst[c] = A.costab[(size_t)L * MAX_L + c];
        snt[c] = A.sintab[(size_t)L * MAX_L + c];
    }
    constexpr double Nd = (double)(L2 * L);
    for (int64_t f = 0; f < nf; ++f) {
        const uint32_t *ra = A.frames + f * A.frame_words + d.frame_off + (size_t)t * L2;
        const uint32_t *rb = ra + (size_t)d.n_T * L2;
        // the frame's two energies, loaded early (used after the plane sums)
        double Ea = 0.0, Eb = 0.0;
        if (tid == NPLANE) {
            const double *E = A.frameE + f * 2 * A.total_slots + 2 * (size_t)d.slot_off;
            Ea = E[t];
            Eb = E[d.n_T + t];
        }
        for (int i = tid; i < L2; i += T) {
            const uint32_t e = ~(ra[i] ^ rb[i]) & mask;
            const int y = i % L, z = i / L;
            eqr[y + LP * z] = e;
            R[y + LP * z] = __builtin_popcount(e);
        }
        __syncthreads();
        column_counts<L>(eqr, tid, C, D);  // C[x][y] at x*LP + y, D[x][z] at x*LP + z
        __syncthreads();
        // plane counts: lane (c, chunk) sums v = chunk, chunk + GC, ... of
        // every family (no divergence: the family loop is unrolled), then
        // (family, c) tasks add the GC chunk partials (integers: any order)
        if (tid < L * GC) {
            const int c = tid % L, chunk = tid / L;
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
                part[fam][chunk][c] = cnt;
            }
        }
        __syncthreads();
        for (int task = tid; task < NPLANE * L; task += T) {
            const int fam = task / L, c = task - fam * L;
            int cnt = 0;
            for (int g = 0; g < GC; ++g) cnt += part[fam][g][c];
            P[fam][c] = 2 * cnt - L2;
        }
        __syncthreads();
        if (tid < NPLANE) {
            double re = 0.0, im = 0.0;
            for (int c = 0; c < L; ++c) {
                re += (double)P[tid][c] * cst[c];
                im += (double)P[tid][c] * snt[c];
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
            int S0 = 0;
            for (int c = 0; c < L; ++c) S0 += P[0][c];
            const double q0 = (double)S0 / Nd;
            accs[0] += 1.0;
            accs[1] += q0;
            accs[2] += q0 * q0;
            accs[3] += (q0 * q0) * q0;
            accs[4] += (q0 * q0) * (q0 * q0);
            accs[32] += Ea;
            accs[33] += Ea * Ea;
            accs[34] += Eb;
            accs[35] += Eb * Eb;
        }
        __syncthreads();
    }
    for (int i = tid; i < NACC; i += T) A.acc[(size_t)gs * NACC + i] = accs[i];
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

// Observables of eqs. 3-6 from disorder-averaged thermal means D[36] (column
// order of the accumulators), each formula evaluated in the order written,
// one rounding per binary64 operation.  two_sin = 2 sin(pi/L) (host libm).
__device__ __forceinline__ void observables_of(const double *D, int L, double two_sin, double *o)
{
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
    o[5] = sqrt(chi0 / chik - 1.0) / two_sin;
    o[6] = chik / chik2;
    o[7] = chi0 / chik;
    o[8] = D[32];
    o[9] = D[34];
}

constexpr int NOBS_VAL = 10;  // observables per slot (the count column aside)

// Disorder averages (eqs. 3-6) and, with jk, leave-one-sample-out jackknife
// errors (Methods, last paragraph) per temperature slot over the S selected
// samples sel[0..S-1] of one system.  One workgroup per slot.
//  1. Column j of the slot: exact sum over samples of the thermal mean
//     acc[j] / acc[0], kept normalized in LDS; D[j] = (rounded sum) / S.
//  2. Observables of D: the central values.
//  3. Replicate s: D_s[j] = (rounded exact sum less sample s's value) / (S-1),
//     observables O_s, kept in rep[t][s][10] (device memory of the caller:
//     nT * S * 10 doubles); exact sums over s of O_s give the replicate mean
//     Obar = (rounded sum) / S, then exact sums of (O_s - Obar)^2 give
//     err = sqrt((S-1)/S * rounded sum).  Each thread reads back only the
//     replicates it wrote.
__global__ void __launch_bounds__(256) finalize_kernel(const SampleDev *samples, const int32_t *sel, int S, int L,
                                                       double two_sin, const double *acc, int jk, double *rep,
                                                       double *mean_out, double *err_out)
{
    __shared__ uint32_t dig[NACC][XL];   // normalized digits of each column's exact sum
    __shared__ int32_t sgn[NACC];        // its final carry (0 or -1)
    __shared__ int32_t spec[NACC][3];    // its NaN, +inf, -inf counts
    __shared__ double D[NACC];
    __shared__ unsigned long long osum[NOBS_VAL][XL];  // exact sums over replicates
    __shared__ int32_t ospec[NOBS_VAL][3];
    __shared__ double obar[NOBS_VAL];
    const int t = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
    if (tid < NACC) {
        int64_t lim[XL];
        for (int k = 0; k < XL; ++k) lim[k] = 0;
        int sp[3] = {0, 0, 0};
        for (int i = 0; i < S; ++i) {
            const double *a = acc + ((size_t)samples[sel[i]].slot_off + t) * NACC;
            const double m = a[tid] / a[0];
            const int c = exact_class(m);
            if (c >= 0) ++sp[c];
            else exact_add(lim, m);
        }
        const int64_t carry = exact_normalize(lim);
        for (int k = 0; k < XL; ++k) dig[tid][k] = (uint32_t)lim[k];
        sgn[tid] = (int32_t)carry;
        for (int c = 0; c < 3; ++c) spec[tid][c] = sp[c];
        double v;
        if (!exact_special(sp[0], sp[1], sp[2], &v)) v = exact_round_normalized(lim, carry);
        D[tid] = v / (double)S;
    }
    __syncthreads();
    if (tid == 0) {
        double o[NOBS_VAL];
        observables_of(D, L, two_sin, o);
        for (int k = 0; k < NOBS_VAL; ++k) mean_out[(size_t)t * (NOBS_VAL + 1) + k] = o[k];
        mean_out[(size_t)t * (NOBS_VAL + 1) + NOBS_VAL] = (double)S;
    }
    if (!jk) return;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = tid; i < NOBS_VAL * XL; i += T) (&osum[0][0])[i] = 0ull;
        for (int i = tid; i < NOBS_VAL * 3; i += T) (&ospec[0][0])[i] = 0;
        __syncthreads();
        for (int i = tid; i < S; i += T) {
            double *ro = rep + ((size_t)t * S + i) * NOBS_VAL;
            double o[NOBS_VAL];
            if (pass == 0) {
                const double *a = acc + ((size_t)samples[sel[i]].slot_off + t) * NACC;
                double Ds[NACC];
                for (int j = 0; j < NACC; ++j) {
                    const double m = a[j] / a[0];
                    const int c = exact_class(m);
                    const int n0 = spec[j][0] - (c == 0), n1 = spec[j][1] - (c == 1), n2 = spec[j][2] - (c == 2);
                    double v;
                    if (!exact_special(n0, n1, n2, &v)) {
                        int64_t lim[XL];
                        for (int k = 0; k < XL; ++k) lim[k] = (int64_t)dig[j][k];
                        lim[XL - 1] += (int64_t)sgn[j] * ((int64_t)1 << 32);
                        if (c < 0) exact_add(lim, m, true);
                        v = exact_round(lim);
                    }
                    Ds[j] = v / (double)(S - 1);
                }
                observables_of(Ds, L, two_sin, o);
                for (int k = 0; k < NOBS_VAL; ++k) ro[k] = o[k];
            } else {
                for (int k = 0; k < NOBS_VAL; ++k) o[k] = ro[k];
            }
            for (int k = 0; k < NOBS_VAL; ++k) {
                double x = o[k];
                if (pass == 1) {
                    const double dv = x - obar[k];
                    x = dv * dv;
                }
                const int c = exact_class(x);
                if (c >= 0) atomicAdd(&ospec[k][c], 1);
                else exact_add_atomic(osum[k], x);
            }
        }
        __syncthreads();
        if (tid < NOBS_VAL) {
            int64_t lim[XL];
            for (int k = 0; k < XL; ++k) lim[k] = (int64_t)osum[tid][k];
            double v;
            if (!exact_special(ospec[tid][0], ospec[tid][1], ospec[tid][2], &v)) v = exact_round(lim);
            if (pass == 0) obar[tid] = v / (double)S;
            else err_out[(size_t)t * (NOBS_VAL + 1) + tid] = sqrt((double)(S - 1) / (double)S * v);
        }
        if (pass == 1 && tid == 0) err_out[(size_t)t * (NOBS_VAL + 1) + NOBS_VAL] = 0.0;
        __syncthreads();
    }
}

}  // namespace ea
