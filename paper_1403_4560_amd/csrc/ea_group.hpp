// ea_group.hpp -- walker-interleaved LDS engine for any even L <= 16 (both
// coupling kinds): the lattice sizes that the row engine (Gaussian L = 8, 16)
// and the one-bit engine (+-1 L = 8, 16, 32) do not take.
//
// Layout: one int8x4 word holds one site of four walkers of a chain (a
// "quad"), [2 parities][quads][N/2 + 1 sites] (the odd plane stride spreads
// the quads of a wave over all LDS banks); a per-item table gives every
// sublattice site its six neighbours in the other sublattice as 16-bit byte
// offsets (both checkerboard offsets for x); a site's six neighbour words and
// six bonds serve four Metropolis attempts at once and the neighbour
// arithmetic works for any L (the four sites of a Philox group may lie in
// different rows).  A work item is (quad, group of four consecutive sublattice
// sites): four Philox calls, one per walker (counter (h >> 2, 2n + p,
// (t << 1) | r, sample), word h & 3, as in every engine), then four word
// updates.  Walkers beyond n_T in the last quad are padding: spins +1, never
// flipped, never tallied.
//
// Device functions only: the per-class kernel (ea_group.hip) and the batch
// kernel (ea_batch.hip) instantiate them.
#pragma once

#include "ea_device.hpp"
#include "ea_item.hpp"
#include "ea_types.hpp"
#include "ea_update.hpp"

namespace ea {

// Neighbours of sublattice site (p, h) in the other sublattice, in the order
// +x, -x, +y, -y, +z, -z.  Site bit k of row (y, z) sits at x = 2k + eps,
// eps = (y + z + p) & 1.
template <int L>
__device__ __forceinline__ void group_nbrs(int p, int h, int nb[6])
{
    constexpr int HL = L / 2;
    const int row = h / HL, k = h - row * HL;
    const int y = row % L, z = row / L;
    const int x = 2 * k + ((y + z + p) & 1);
    const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
    const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
    const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
    nb[0] = (xp >> 1) + HL * row;
    nb[1] = (xm >> 1) + HL * row;
    nb[2] = k + HL * (yp + L * z);
    nb[3] = k + HL * (ym + L * z);
    nb[4] = k + HL * (y + L * zp);
    nb[5] = k + HL * (y + L * zm);
}

// Word of (parity p, sublattice site h, quad q).
template <int L>
__device__ __forceinline__ int gidx(int p, int h, int q, int NQ)
{
    constexpr int PS = L * L * L / 2 + 1;
    return (p * NQ + q) * PS + h;
}

// Neighbour table entry of sublattice site h, stored at (h & 3) N/8 + h / 4
// (the lanes of a wave read one site of consecutive site groups: contiguous
// 16-byte entries, free of bank conflicts): the byte offsets 4 n of its
// neighbour words (and of their int32 bonds) in 16-bit halves, {+y | -y << 16,
// +z | -z << 16, +x | -x << 16 for parity 0, the same for parity 1}, so that
// an address is one add of a half-word to a base (4 n < 2^16 for L <= 16).
template <int L>
__device__ __forceinline__ uint4 nbr_entry(int h)
{
    static_assert(2 * L * L * L < 65536, "byte offsets must fit 16 bits");
    int n0[6], n1[6];
    group_nbrs<L>(0, h, n0);
    group_nbrs<L>(1, h, n1);
    return make_uint4((uint32_t)(4 * n0[2]) | (uint32_t)(4 * n0[3]) << 16,
                      (uint32_t)(4 * n0[4]) | (uint32_t)(4 * n0[5]) << 16,
                      (uint32_t)(4 * n0[0]) | (uint32_t)(4 * n0[1]) << 16,
                      (uint32_t)(4 * n1[0]) | (uint32_t)(4 * n1[1]) << 16);
}

struct GroupLane {
    float ka[4], kb[4];     // per walker: the folded exponent's constants (update_word_gauss)
    uint32_t c2[4];         // Philox counter word 2 of each walker
    uint32_t thr[4];        // +-1: offset of each walker's threshold table in lut
    uint32_t valid;         // 0xFF in the bytes of real walkers
    float h32;              // the sample's field, held in a vector register
};

struct GroupTally {
    uint32_t flips = 0;     // per byte: flipped sites of that walker
    uint32_t fdown = 0;     // per byte: flipped sites that were -1
    uint32_t nd = 0;        // per byte, second half: -1 spins after the update
    int accE[4] = {0, 0, 0, 0};  // second half: sum of (S_u + hgrid) XOR m' per walker (Gaussian)
};

// Metropolis update of work item (quad q, sites 4 g4 .. 4 g4 + 3) of parity P.
template <int L, int JK, int P>
__device__ __forceinline__ void group_item(const SweepArgs &A, const SampleDev &d, uint32_t *SG, const void *Jl,
                                           const uint32_t *lut, const float *b32, const uint4 *NB, int NQ, int q,
                                           int g4, uint32_t c1, const GroupLane &ln, GroupTally &ty)
{
    constexpr int HALF = L * L * L / 2, PS = HALF + 1;
    uint32_t *Sp = SG + (P * NQ + q) * PS;
    const uint32_t *So = SG + ((1 - P) * NQ + q) * PS;
    u32x4 rw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) rw[i] = philox4x32_10((uint32_t)g4, c1, ln.c2[i], d.sample_id, A.key0, A.key1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int h = 4 * g4 + k;
        const uint4 te = NB[k * (HALF / 4) + g4];
        const uint32_t tx = P ? te.w : te.z;
        const uint32_t off[6] = {tx & 0xFFFFu, tx >> 16, te.x & 0xFFFFu, te.x >> 16, te.y & 0xFFFFu, te.y >> 16};
        const uint32_t Sv = Sp[h];
        uint32_t X[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) X[j] = *(const uint32_t *)((const char *)So + off[j]);
        const u32x4 rk = {k == 0 ? rw[0].x : k == 1 ? rw[0].y : k == 2 ? rw[0].z : rw[0].w,
                          k == 0 ? rw[1].x : k == 1 ? rw[1].y : k == 2 ? rw[1].z : rw[1].w,
                          k == 0 ? rw[2].x : k == 1 ? rw[2].y : k == 2 ? rw[2].z : rw[2].w,
                          k == 0 ? rw[3].x : k == 1 ? rw[3].y : k == 2 ? rw[3].z : rw[3].w};
        uint32_t fm;
        int Sus[4];
        if constexpr (JK == 0) {
            // bonds +x, -x, +y, -y, +z, -z: own +d bonds, the neighbours' +d bonds for -d
            const int *Jp = (const int *)Jl + (size_t)P * 3 * HALF, *Jo = (const int *)Jl + (size_t)(1 - P) * 3 * HALF;
            const char *Jb = (const char *)Jo;
            const int jx = Jp[h], jxm = *(const int *)(Jb + off[1]), jy = Jp[HALF + h];
            const int jym = *(const int *)(Jb + 4 * HALF + off[3]);
            const int jz = Jp[2 * HALF + h], jzm = *(const int *)(Jb + 8 * HALF + off[5]);
            const int Ja[4] = {jx, jx, jx, jx}, Js[4] = {jxm, jxm, jxm, jxm};
            const int Jy[4] = {jy, jy, jy, jy}, Jyn[4] = {jym, jym, jym, jym};
            const int Jz[4] = {jz, jz, jz, jz}, Jzn[4] = {jzm, jzm, jzm, jzm};
            // the exact path reads 2 beta32 of walker i's slot, t = bits 1 .. 27 of its counter word
            // Sus = S_u + hgrid (the field's grid part folded into the integer field)
            fm = update_word_gauss<true>(Sv, X[0], X[1], X[2], X[3], X[4], X[5], Ja, Js, Jy, Jyn, Jz, Jzn, rk,
                                         ln.ka, ln.kb, [&](int i) { return 2.0f * b32[(ln.c2[i] >> 1) & 0x7FFFFFFu]; },
                                         ln.h32, d.hgrid, Sus) &
                 ln.valid;
        } else {
            // bond-spin product bytes J s_j: 0x01 (+1) or 0xFF (-1); c counts the -1
            const int8_t *Jp = (const int8_t *)Jl + (size_t)P * 3 * HALF;
            const int8_t *Jo = (const int8_t *)Jl + (size_t)(1 - P) * 3 * HALF;
            const int8_t jb[6] = {Jp[h], Jo[off[1] >> 2], Jp[HALF + h], Jo[HALF + (off[3] >> 2)], Jp[2 * HALF + h],
                                  Jo[2 * HALF + (off[5] >> 2)]};
            constexpr uint32_t LOW = 0x01010101u;
            uint32_t cnt = 0;
#pragma unroll
            for (int j = 0; j < 6; ++j) cnt += ((X[j] ^ (jb[j] < 0 ? 0xFEFEFEFEu : 0u)) >> 7) & LOW;
            const uint32_t words[4] = {rk.x, rk.y, rk.z, rk.w};
            fm = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int sh = 8 * i;
                const int b = 6 - (int)((cnt >> sh) & 0xFFu);               // (S_J + 6) / 2
                const int m = __builtin_amdgcn_sbfe((int)Sv, sh + 7, 1);  // 0: s_i = +1, -1: s_i = -1
                const int idx = (m + 1) * 7 + b;
                Sus[i] = 2 * b - 6;  // S_J
                const bool accept = ((d.down_mask >> idx) & 1u) | (words[i] < lut[ln.thr[i] + idx]);
                fm |= accept ? 0xFEu << sh : 0u;
            }
            fm &= ln.valid;
        }
        Sp[h] = Sv ^ fm;
        ty.flips += (fm >> 7) & 0x01010101u;
        ty.fdown += ((fm & Sv) >> 7) & 0x01010101u;
        if constexpr (P == 1) {
            const uint32_t Sn = Sv ^ fm;
#pragma unroll
            for (int i = 0; i < 4; ++i) ty.accE[i] += Sus[i] ^ __builtin_amdgcn_sbfe((int)Sn, 8 * i + 7, 1);
            ty.nd += (Sn >> 7) & 0x01010101u;
        }
    }
}

template <int L, int JK>
__device__ __forceinline__ void run_group_item(const SweepArgs &A, const SampleDev &d, int r, char *smem,
                                               const Team tm = whole_block())
{
    constexpr int N = L * L * L, HALF = N / 2, G4 = HALF / 4;
    const int nT = d.n_T, NQ = (nT + 3) / 4;
    const int T = tm.T, tid = tm.tid;
    const GroupLdsOff o = group_lds_offsets(L, nT, JK);
    uint32_t *SG = (uint32_t *)(smem + o.spins);
    void *Jl = (void *)(smem + o.J);
    uint32_t *lut = (uint32_t *)(smem + o.lut);
    uint4 *NB = (uint4 *)(smem + o.nb);
    ItemLds I{};
    I.was = (int32_t *)(smem + o.was);
    I.sow = (int32_t *)(smem + o.sow);
    I.M = (int32_t *)(smem + o.M);
    I.dM = (int32_t *)(smem + o.dM);
    I.fl = (int32_t *)(smem + o.fl);
    I.sw = (int32_t *)(smem + o.sw);
    I.EJ = (long long *)(smem + o.EJ);
    I.dEJ = (long long *)(smem + o.dEJ);
    I.b32 = (float *)(smem + o.b32);
    I.b64 = (double *)(smem + o.b64);

    const size_t sbase = (size_t)d.spin_off + (size_t)r * nT * N;
    const int gi = 2 * d.slot_off + r * nT;
    // spins: int8 [walker][parity][N/2] -> quad words
    for (int j = tid; j < 2 * HALF * NQ; j += T) {
        const int q = j % NQ, ph = j / NQ;
        uint32_t wv = 0;
        for (int i = 0; i < 4; ++i) {
            const int w = 4 * q + i;
            const uint32_t b = w < nT ? (uint32_t)(uint8_t)A.spins[sbase + (size_t)w * N + ph] : 0x01u;
            wv |= b << (8 * i);
        }
        SG[gidx<L>(ph / HALF, ph % HALF, q, NQ)] = wv;
    }
    for (int h = tid; h < HALF; h += T) NB[(h & 3) * G4 + (h >> 2)] = nbr_entry<L>(h);
    if constexpr (JK == 0) {
        // couplings as exact int32 multiples of 2^-18
        const float4 *src = (const float4 *)((const float *)A.J + d.J_off);  // J_off is a multiple of 4
        int4 *dst = (int4 *)Jl;
        for (int i = tid; i < 3 * N / 4; i += T) {
            const float4 v = src[i];
            dst[i] = make_int4((int)(v.x * 262144.0f), (int)(v.y * 262144.0f), (int)(v.z * 262144.0f),
                               (int)(v.w * 262144.0f));
        }
    } else {
        block_copy(Jl, (const int8_t *)A.J + d.J_off, (size_t)3 * N, tm);
        for (int i = tid; i < nT * 14; i += T) lut[i] = A.lut[(size_t)d.slot_off * 14 + i];
    }
    for (int i = tid; i < nT; i += T) {
        I.was[i] = A.was[gi + i];
        I.sow[A.was[gi + i]] = i;  // kept by exchange_pass from here on
        // walker totals: E_J = -dEJ, magnetisation M + dM (see the sweep loop)
        I.dEJ[i] = -A.EJ[gi + i];
        I.dM[i] = 0;
        I.M[i] = A.M[gi + i];
        I.fl[i] = 0;
        I.sw[i] = 0;
        I.b32[i] = A.beta32[d.slot_off + i];
        I.b64[i] = A.beta[d.slot_off + i];
    }
    // padding walkers of the last quad read slot 0's constants (never used:
    // their bytes are never flipped or tallied)
    for (int i = nT + tid; i < 4 * NQ; i += T) I.sow[i] = 0;
    __syncthreads();

    // thread -> (quad, first site group); threads beyond NQ * TPQ stay idle.
    // A team of eight waves holds two per SIMD (waves w and w + 4 share one;
    // the order of the four SIMDs varies by workgroup).  When the site groups
    // do not divide evenly (L = 12: 864 items on 512 threads, five and a half
    // waves take two groups per half-sweep), those waves are placed by SIMD:
    // both waves of SIMDs 2p and 2p+1 and one wave of each other SIMD, p the
    // parity of blockIdx / 256 (the two workgroups of a CU start 256 blocks
    // apart), so that together the two load the CU's four SIMDs evenly.  The
    // SIMD of each wave is read from the HW_ID register and exchanged through
    // the frame's EJ array, which this engine does not otherwise use (at least
    // 32 bytes).  Results do not depend on the placement.
    int vt = tid;
    if (T == 512 && 64 % NQ == 0) {
        int *wave_simd = (int *)(smem + o.EJ);
        if ((tid & 63) == 0) wave_simd[tid >> 6] = (int)__builtin_amdgcn_s_getreg((1 << 11) | (4 << 6) | 4) & 3;
        __syncthreads();
        int n_on[4] = {0, 0, 0, 0};
        for (int k = 0; k < 8; ++k) n_on[wave_simd[k]]++;
        if (n_on[0] == 2 && n_on[1] == 2 && n_on[2] == 2 && n_on[3] == 2) {
            const int w = tid >> 6, sm = wave_simd[w], p = (blockIdx.x >> 8) & 1;
            int rank = 0;  // 0 for the first of the SIMD's two waves, 1 for the second
            for (int k = 0; k < w; ++k) rank += wave_simd[k] == sm;
            const int role = (sm >> 1) == p ? 2 * (sm & 1) + rank : 4 + (sm & 1) + 2 * rank;
            vt = role * 64 + (tid & 63);
        }
    }
    const int TPQ = T / NQ;
    const int q = vt % NQ, gs = vt / NQ;
    const bool on = gs < TPQ;
    uint32_t valid = 0;
    for (int i = 0; i < 4; ++i) valid |= (4 * q + i < nT ? 0xFFu : 0u) << (8 * i);
    const double unit = JK == 0 ? 0x1p-18 : 1.0;
    const double hd = (double)d.h32;
    const int hg = JK == 0 ? d.hgrid : 0;  // the field's grid part folded into S_u
    const int64_t n0 = A.state[0];
    int64_t next_meas = next_measurement(n0, A.measure_every, A.measure_start);
    int64_t f = 0;  // frame of the next measurement within this chunk
    // Energy of walker w after a sweep: its second half-sweep's tallies leave
    // minus E_J in dEJ and the magnetisation change in dM; both are folded in
    // at the start of the next sweep, before its own tallies (which follow the
    // first half-sweep's barrier), so no pass of their own is needed.
    const auto energy = [&](int w) { return (double)(-I.dEJ[w]) * unit - hd * (double)(I.M[w] + I.dM[w]); };
    for (int it = 0; it < A.K; ++it) {
        const int64_t n = n0 + it;
#pragma unroll 1
        for (int i = tid; i < nT; i += T) {
            I.M[i] += I.dM[i];
            I.dM[i] = 0;
            I.dEJ[i] = -(long long)hg * HALF;
        }
        GroupLane ln;
        int ts[4];
        for (int i = 0; i < 4; ++i) {
            const int w = 4 * q + i;
            ts[i] = I.sow[w];  // (padding walkers: slot 0)
            const float cp = two_beta_log2e(I.b32[ts[i]]);
            ln.ka[i] = cp * 0x1p-18f;
            ln.kb[i] = cp * (d.h32 - (float)d.hgrid * 0x1p-18f);
            ln.c2[i] = (PURPOSE_METROPOLIS << 28) | ((uint32_t)ts[i] << 1) | (uint32_t)r;
            ln.thr[i] = 14 * ts[i];
        }
        ln.valid = valid;
        ln.h32 = d.h32;
        asm volatile("" : "+v"(ln.h32));
        GroupTally ty;
        if (on) {
            const uint32_t c1 = (uint32_t)(2 * n);
#pragma unroll 1
            for (int g4 = gs; g4 < G4; g4 += TPQ)
                group_item<L, JK, 0>(A, d, SG, Jl, lut, I.b32, NB, NQ, q, g4, c1, ln, ty);
        }
        __syncthreads();
        if (on) {
            const uint32_t c1 = (uint32_t)(2 * n + 1);
#pragma unroll 1
            for (int g4 = gs; g4 < G4; g4 += TPQ)
                group_item<L, JK, 1>(A, d, SG, Jl, lut, I.b32, NB, NQ, q, g4, c1, ln, ty);
        }
        // Per-walker tallies (idle lanes hold zeros).  dEJ collects minus the
        // new E_J: the second half-sweep summed (S_u + hgrid) XOR m' = s'(S_u +
        // hgrid) - [s' = -1] over the odd sites, so a thread adds accE +
        // (1 + 2 hgrid) nd and dEJ starts the sweep at -hgrid N/2 (+-1
        // couplings: hgrid = 0).  Per thread a byte counter holds at most 128
        // (at most 16 site groups per half-sweep), so a sum over 16 lanes fits
        // a 16-bit lane.  Teams of four or more waves with NQ = 1, 2 or 4 sum
        // the lanes of a row of 16 that share a quad (lane = quad mod NQ)
        // first (byte counters as 16-bit lanes, walkers 0 and 2 in one word,
        // 1 and 3 in another); lane j of the row then adds walker (j / NQ) mod
        // 4 of quad j mod NQ, so a wave issues three LDS atomics, not twelve.
        // With NQ = 4 and at most five site groups per thread and half-sweep
        // (any team size), the four lanes of a quad's residue class sum in
        // narrower words: byte counters stay bytes (at most 4 x 2 x 4 x 5 =
        // 160 flips) and the energy tallies stay int32 (at most 4 x 4 x 5 = 80
        // sites of |(S_u + hgrid) XOR m'| <= 12 2^21 + 1, below 2^31).
        const int hg1 = 2 * hg + 1;  // |hgrid| <= 6 2^21
        if (NQ == 4 && 5 * TPQ >= G4) {
            int cf = (int)ty.flips, cd = (int)ty.fdown, cn = (int)ty.nd;
            cf += row_rotate<4>(cf);
            cd += row_rotate<4>(cd);
            cn += row_rotate<4>(cn);
            cf += row_rotate<8>(cf);
            cd += row_rotate<8>(cd);
            cn += row_rotate<8>(cn);
            int e[4];
            for (int i = 0; i < 4; ++i) {
                e[i] = ty.accE[i];
                e[i] += row_rotate<4>(e[i]);
                e[i] += row_rotate<8>(e[i]);
            }
            int tl = tid;
            asm volatile("" : "+v"(tl));
            const int sel = (tl >> 2) & 3, w = 4 * (tl & 3) + sel, sh = 8 * sel;
            const int fl = (int)(((uint32_t)cf >> sh) & 0xFFu);
            const int fd = (int)(((uint32_t)cd >> sh) & 0xFFu);
            const int nd = (int)(((uint32_t)cn >> sh) & 0xFFu);
            const int ea = sel == 0 ? e[0] : sel == 1 ? e[1] : sel == 2 ? e[2] : e[3];
            const int t = sel == 0 ? ts[0] : sel == 1 ? ts[1] : sel == 2 ? ts[2] : ts[3];
            if (w < nT) {
                atomicAdd((unsigned long long *)&I.dEJ[w], (unsigned long long)((long long)ea + (long long)hg1 * nd));
                atomicAdd(&I.dM[w], -2 * (fl - 2 * fd));
                atomicAdd(&I.fl[t], fl);
            }
        } else if (T >= 256 && NQ <= 4 && NQ != 3) {
            uint32_t c[6] = {ty.flips & 0x00FF00FFu, (ty.flips >> 8) & 0x00FF00FFu,
                             ty.fdown & 0x00FF00FFu, (ty.fdown >> 8) & 0x00FF00FFu,
                             ty.nd & 0x00FF00FFu,    (ty.nd >> 8) & 0x00FF00FFu};
            for (int k = 0; k < 6; ++k) c[k] = (uint32_t)row_residue_sum((int)c[k], NQ);
            long long e[4];
            for (int i = 0; i < 4; ++i) e[i] = row_residue_sum((long long)ty.accE[i], NQ);
            // (lane roles from an opaque copy of the thread index: derived per
            // sweep, not hoisted out of the item loop and spilled)
            int tl = tid;
            asm volatile("" : "+v"(tl));
            // (NQ = 1, 2, 4: j / NQ = j >> (NQ >> 1))
            const int j = tl & 15, sel = (j >> (NQ >> 1)) & 3, w = 4 * (tl & (NQ - 1)) + sel, sh = 16 * (sel >> 1);
            const bool odd = sel & 1;
            const int fl = (int)(((odd ? c[1] : c[0]) >> sh) & 0xFFFFu);
            const int fd = (int)(((odd ? c[3] : c[2]) >> sh) & 0xFFFFu);
            const int nd = (int)(((odd ? c[5] : c[4]) >> sh) & 0xFFFFu);
            const long long ea = sel == 0 ? e[0] : sel == 1 ? e[1] : sel == 2 ? e[2] : e[3];
            const int t = sel == 0 ? ts[0] : sel == 1 ? ts[1] : sel == 2 ? ts[2] : ts[3];
            if (j < 4 * NQ && w < nT) {
                atomicAdd((unsigned long long *)&I.dEJ[w], (unsigned long long)(ea + (long long)hg1 * nd));
                atomicAdd(&I.dM[w], -2 * (fl - 2 * fd));
                atomicAdd(&I.fl[t], fl);
            }
        } else {
            for (int i = 0; i < 4; ++i) {
                const int w = 4 * q + i;
                if (w < nT) {
                    const int fl = (int)((ty.flips >> (8 * i)) & 0xFFu), fd = (int)((ty.fdown >> (8 * i)) & 0xFFu);
                    const int nd = (int)((ty.nd >> (8 * i)) & 0xFFu);
                    atomicAdd((unsigned long long *)&I.dEJ[w], (unsigned long long)(ty.accE[i] + (long long)hg1 * nd));
                    atomicAdd(&I.dM[w], -2 * (fl - 2 * fd));
                    atomicAdd(&I.fl[ts[i]], fl);
                }
            }
        }
        __syncthreads();
        exchange_pass_e(A, d, r, n, I, energy, tm);
        __syncthreads();
        // Snapshot for the overlap measurement, in slot order.
        const int64_t done = n + 1;
        if (done == next_meas) {
            next_meas += A.measure_every;
            uint32_t *dst = A.frames + f * A.frame_words + d.frame_off + (size_t)r * nT * L * L;
            // One (quad, row) per step: the row's L words hold the four walkers'
            // spins; their sign bits, moved to bit 0 of each byte and shifted by
            // x, build the four walkers' rows at once (byte b of lo: x < 8, of
            // hi: x >= 8).  Site x of row (y, z) is sublattice site
            // row L/2 + x/2 of parity (x + y + z) & 1.
            constexpr int HL = L / 2, PS = HALF + 1;
            for (int i = tid; !tm.ghost && i < NQ * L * L; i += T) {
                const int q = i / (L * L), row = i - q * (L * L);
                const int e = ((row % L) + row / L) & 1;  // parity of the even x
                const uint32_t *ev = SG + (e * NQ + q) * PS + row * HL;
                const uint32_t *od = SG + ((1 - e) * NQ + q) * PS + row * HL;
                uint32_t lo = 0, hi = 0;
#pragma unroll
                for (int x = 0; x < L; ++x) {
                    const uint32_t sg = (((x & 1) ? od : ev)[x >> 1] >> 7) & 0x01010101u;
                    if (x < 8) lo |= sg << x;
                    else hi |= sg << (x - 8);
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int w = 4 * q + b;
                    if (w < nT) dst[I.sow[w] * L * L + row] = ((lo >> (8 * b)) & 0xFFu) | (((hi >> (8 * b)) & 0xFFu) << 8);
                }
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
    for (int j = tid; !tm.ghost && j < 2 * HALF * NQ; j += T) {
        const int q2 = j % NQ, ph = j / NQ;
        const uint32_t wv = SG[gidx<L>(ph / HALF, ph % HALF, q2, NQ)];
        for (int i = 0; i < 4; ++i) {
            const int w = 4 * q2 + i;
            if (w < nT) A.spins[sbase + (size_t)w * N + ph] = (int8_t)((wv >> (8 * i)) & 0xFFu);
        }
    }
    for (int i = tid; !tm.ghost && i < nT; i += T) {
        A.was[gi + i] = I.was[i];
        A.EJ[gi + i] = -I.dEJ[i];
        A.M[gi + i] = I.M[i] + I.dM[i];
        A.flips[gi + i] += I.fl[i];
        A.swaps[gi + i] += I.sw[i];
    }
    __syncthreads();
}

}  // namespace ea
