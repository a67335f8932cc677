// ea_row.hpp -- the per-item frame of the byte-per-spin LDS engines (one
// (sample, chain) work item held in LDS for a chunk of sweeps) with its two
// half-sweep engines: the row engine (L = 8, 16, Gaussian couplings; int8x4
// words of four sites of one walker) and the site engine (any even L <= 16,
// either coupling kind; one site at a time).  Device functions only: the
// per-class kernels (ea_kernels.hip) and the batch kernel (ea_batch.hip)
// instantiate them.
#pragma once

#include "ea_device.hpp"
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
                                                int64_t n, const ItemLds &I, const Team tm)
{
    constexpr int N = L * L * L, HALF = N / 2, G = HALF / 4, HL = L / 2;
    const int nT = d.n_T;
    const int T = tm.T, tid = tm.tid;
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
__device__ __forceinline__ void run_item(const SweepArgs &A, const SampleDev &d, int r, char *smem,
                                         const Team tm = whole_block())
{
    constexpr int N = L * L * L;
    const int nT = d.n_T;
    const int T = tm.T, tid = tm.tid;
    const ItemLds I = item_lds(smem, L, nT, JK);

    const size_t sbase = (size_t)d.spin_off + (size_t)r * nT * N;
    const int gi = 2 * d.slot_off + r * nT;
    copy_walkers(I.S, item_walker_stride(L), A.spins + sbase, nT, N, true, tm);
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
                   (size_t)3 * N * (JK == 0 ? 4 : 1), tm);
    }
    for (int i = tid; i < nT; i += T) {
        I.was[i] = A.was[gi + i];
        I.sow[A.was[gi + i]] = i;  // kept by exchange_pass from here on
        // row engine: E_J = -dEJ (see the sweep loop); site engine: EJ + dEJ
        I.dEJ[i] = ROW ? -A.EJ[gi + i] : 0;
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
    // (from an opaque copy of the thread index: derived here, after the loads,
    // not hoisted to the kernel's start and kept across them, which spills)
    int tid_r = tid;
    asm volatile("" : "+v"(tid_r));
    const int rw_wave = tid_r >> 6, rw_lane = tid_r & 63;
    const int rw_par = __builtin_amdgcn_readfirstlane(rw_wave & 1);
    const int rw_rem = rw_lane % CPW;
    const int rw_w = (rw_wave >> 1) * WPW + rw_lane / CPW;
    const int rw_k = rw_rem % WPR, rw_y = 2 * (rw_rem / WPR) + rw_par;

    const double unit = JK == 0 ? 0x1p-18 : 1.0;
    const double hd = (double)d.h32;
    const int64_t n0 = A.state[0];
    // (the period from an opaque copy: the division's set-up is then made
    // here, per item, rather than hoisted out of the item loop of a
    // persistent kernel and held in registers across it, which spills)
    int32_t every = A.measure_every;
    asm volatile("" : "+s"(every));
    int64_t next_meas = next_measurement(n0, every, A.measure_start);
    int64_t f = 0;  // frame of the next measurement within this chunk
    // Energy of walker w after a sweep.  Row engine: the second half-sweep's
    // tallies leave minus E_J in dEJ and the magnetisation change in dM; both
    // are folded in at the start of the next sweep, before its own tallies
    // (which follow the first half-sweep's barrier), so no pass of their own
    // is needed.  Site engine: a pass after the sweep folds them in.
    const auto energy = [&](int w) {
        return ROW ? (double)(-I.dEJ[w]) * unit - hd * (double)(I.M[w] + I.dM[w])
                   : (double)I.EJ[w] * unit - hd * (double)I.M[w];
    };
    for (int it = 0; it < A.K; ++it) {
        const int64_t n = n0 + it;
        if constexpr (ROW) {
#pragma unroll 1
            for (int i = tid; i < nT; i += T) {
                I.M[i] += I.dM[i];
                I.dM[i] = 0;
                I.dEJ[i] = 0;
            }
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
                // leaves sum s' S_u, at most 4 L x 6 2^21 in size per thread:
                // a group of four threads (L = 8) sums it in int32 (128 sites
                // x 6 2^21 < 2^31), a row of sixteen (L = 16) in int64.
                const long long own = (long long)accE + nd - (long long)d.hgrid * (4 * L - 2 * nd);
                long long sE;
                if constexpr (CPW == 4) sE = group_sum_dpp<CPW>((int)own);
                else sE = group_sum_dpp<CPW>(own);
                const int sf = group_sum_dpp<CPW>(bf), sd = group_sum_dpp<CPW>(bd);
                if (rw_rem == 0) {
                    const int flips = (int)((unsigned)sf / 7u), ndown = (int)((unsigned)sd / 7u);
                    // dEJ collects minus the new E_J (both waves of the walker add)
                    atomicAdd((unsigned long long *)&I.dEJ[rw_w], (unsigned long long)sE);
                    atomicAdd(&I.dM[rw_w], -2 * (flips - 2 * ndown));
                    atomicAdd(&I.fl[t], flips);
                }
            }
        } else {
            site_half_sweep<L, JK>(A, d, r, 0, n, I, tm);
            __syncthreads();
            site_half_sweep<L, JK>(A, d, r, 1, n, I, tm);
        }
        __syncthreads();
        if constexpr (!ROW) {
            for (int i = tid; i < nT; i += T) {
                I.EJ[i] += I.dEJ[i];
                I.M[i] += I.dM[i];
                I.dEJ[i] = 0;  // cleared for the next sweep's tallies
                I.dM[i] = 0;
            }
            __syncthreads();
        }
        exchange_pass_e(A, d, r, n, I, energy, tm);
        __syncthreads();
        // Snapshot for the overlap measurement, in slot order.
        const int64_t done = n + 1;
        if (done == next_meas) {
            next_meas += A.measure_every;
            uint32_t *dst = A.frames + f * A.frame_words + d.frame_off + (size_t)r * nT * L * L;
            for (int i = tid; !tm.ghost && i < nT * L * L; i += T) {
                const int t = i / (L * L), row = i - t * (L * L);
                dst[i] = pack_row_lds<L>(I.S + (size_t)I.was[t] * item_walker_stride(L), row);
            }
            for (int t = tid; !tm.ghost && t < nT; t += T) {
                const int w = I.was[t];
                A.frameE[f * 2 * A.total_slots + gi + t] = energy(w);
            }
            ++f;
            __syncthreads();  // the next sweep changes the spins read here
        }
    }
    __syncthreads();
    // Write-back addresses are derived again from an opaque copy of the thread
    // index rather than kept from the load phase: held across the sweep loop
    // they would be spilled to scratch memory (the L = 16 row kernel uses
    // every register it may have).
    Team tw = tm;
    asm volatile("" : "+v"(tw.tid));
    if (!tw.ghost) copy_walkers(I.S, item_walker_stride(L), A.spins + sbase, nT, N, false, tw);
    for (int i = tw.tid; !tw.ghost && i < nT; i += T) {
        A.was[gi + i] = I.was[i];
        A.EJ[gi + i] = ROW ? -I.dEJ[i] : I.EJ[i];
        A.M[gi + i] = ROW ? I.M[i] + I.dM[i] : I.M[i];
        A.flips[gi + i] += I.fl[i];
        A.swaps[gi + i] += I.sw[i];
    }
    __syncthreads();
}

}  // namespace ea
