// ea_bits.hip -- multispin-coded LDS engine for +-1 couplings (L = 8, 16, 32).
//
// The paper's own GPU kernel packs spins one bit each (Methods: multispin
// coding); this engine does the same on gfx950.  A (sample, chain) work item
// keeps its n_T walkers as bits in LDS -- 4 KB per walker at L = 32, so a
// whole 32-temperature chain (128 KB) plus its bond bits (24 KB) fits in one
// CU's 160 KB -- for a chunk of sweeps, with the same per-sweep frame as the
// byte engines: two checkerboard half-sweeps, exact energies, the replica
// exchange, snapshots for the overlap measurement.
//
// Word layout: bit j of word g of sublattice p holds the site with sublattice
// index h = 32 g + j (bit set iff the spin is -1).  A sublattice row (y, z)
// holds L/2 consecutive indices, so a word holds R = 64/L whole rows of one
// z plane (L = 8: the whole plane).  Site bit k of row (y, z) sits at
// x = 2k + eps, eps = (y + z + p) & 1; its x neighbours in the other
// sublattice are bit k ("aligned") and bit k + 1 (eps = 1) or k - 1 (eps = 0)
// of the same row, cyclic within the row; the y neighbours are the adjacent
// rows (a funnel shift across two words), the z neighbours the words one
// plane away.
//
// Per word (32 sites, one walker): a bond is unsatisfied (J s_i s_j = -1) iff
// the XOR of its three bits is 1; the count c of unsatisfied bonds of every
// site is formed bit-sliced (two full adders and a carry-save step), so the
// local field is S_J = 6 - 2c for s_i = +1 and 2c - 6 for s_i = -1.  The
// contract's acceptance (dE <= 0, or w < thr[t][a][b], a = (s+1)/2,
// b = (S_J + 6)/2) splits into two parts.  dE <= 0 holds iff c >= k_s for a
// threshold k_s per spin sign (the field rises monotonically with c),
// evaluated bit-sliced as the borrow of c - k_s.  The other sites need the
// table entry of their class (s_i, c) with c < k_s; since k_+ + k_- <= 8,
// e = c for s = -1 and e = 7 - c for s = +1 numbers those classes without
// collision in three bits (e = c XOR 7 when s = +1), and a 256-entry LDS
// table spreads the three bit planes of e into bytes that address the slot's
// 8-entry threshold table directly.
// Each site still draws its own Philox word: counter (h >> 2, 2n + p,
// (t << 1) | r, sample), word h & 3, as in every engine.
#include "ea_device.hpp"
#include "ea_item.hpp"
#include "ea_types.hpp"

namespace ea {

__host__ __device__ constexpr uint32_t rep_bit(int seg, int b)
{
    uint32_t m = 0;
    for (int r = 0; r < 32 / seg; ++r) m |= 1u << (r * seg + b);
    return m;
}

__host__ __device__ constexpr uint32_t even_rows(int seg)
{
    uint32_t m = 0;
    for (int r = 0; r < 32 / seg; r += 2) m |= ((1u << seg) - 1u) << (r * seg);
    return m;
}

template <int L>
struct BitGeo {
    static constexpr int N = L * L * L, HALF = N / 2, G = HALF / 32;
    static constexpr int SEG = L / 2;   // sites of one sublattice row
    static constexpr int R = 32 / SEG;  // rows per word
    static constexpr int WPP = L / R;   // words per z plane
    static constexpr uint32_t TOP = rep_bit(SEG, SEG - 1), BOT = rep_bit(SEG, 0), EVEN = even_rows(SEG);
};

__device__ __forceinline__ uint32_t sel(uint32_t a, uint32_t b, uint32_t m) { return (a & ~m) | (b & m); }
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);  // truth table of the majority
}
// Spreading table and threshold tables sit at fixed LDS offsets, ahead of the
// spins: byte addresses then come straight from the spread bytes.
constexpr int SPREAD_OFF = 0, TH_OFF = 256 * 8;

// 2 F + (a < b): the comparison's carry goes straight into the add.
__device__ __forceinline__ uint32_t shift_in_less(uint32_t F, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_cmp_lt_u32_e32 vcc, %1, %2\n\tv_addc_co_u32_e32 %0, vcc, %3, %3, vcc"
        : "=v"(r)
        : "v"(a), "v"(b), "v"(F)
        : "vcc");
    return r;
}

// Loads from an LDS byte address.
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
typedef __attribute__((address_space(3))) const uint64_t lds_u64;
__device__ __forceinline__ uint32_t lds_load(uint32_t addr) { return *(lds_u32 *)(size_t)addr; }
__device__ __forceinline__ uint2 lds_load2(uint32_t addr)
{
    const uint64_t v = *(lds_u64 *)(size_t)addr;
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}
__device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)(size_t)(__attribute__((address_space(3))) const char *)p;
}

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, int s)
{
    return __builtin_amdgcn_alignbit(hi, lo, s);  // ({hi, lo} >> s) low word
}

// Spin bits of 32 int8 spins (bit b set iff byte b is -1) and back.
__device__ __forceinline__ uint32_t pack4(uint32_t v)
{
    return ((v >> 7) & 1u) | ((v >> 14) & 2u) | ((v >> 21) & 4u) | ((v >> 28) & 8u);
}
__device__ __forceinline__ uint32_t unpack4(uint32_t nib)
{
    return 0x01010101u + ((nib * 0x00204081u) & 0x01010101u) * 0xFEu;  // bytes 0x01 / 0xFF
}

// Row bits of one sublattice row spread to the even bit positions.
__device__ __forceinline__ uint32_t spread2(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Bytes 8M .. 8M + 7 of the class planes spread to byte offsets 4 e (sites
// 8M .. 8M + 3 in Q[2M], 8M + 4 .. 8M + 7 in Q[2M + 1]); sp = LDS address of
// the spreading table.
template <int M>
__device__ __forceinline__ void spread3(uint32_t sp, uint32_t E0, uint32_t E1, uint32_t E2, uint32_t Q[8])
{
    const uint2 t0 = lds_load2(sp + 8 * ((E0 >> (8 * M)) & 0xFFu));
    const uint2 t1 = lds_load2(sp + 8 * ((E1 >> (8 * M)) & 0xFFu));
    const uint2 t2 = lds_load2(sp + 8 * ((E2 >> (8 * M)) & 0xFFu));
    Q[2 * M] = t0.x | (t1.x << 1) | (t2.x << 2);
    Q[2 * M + 1] = t0.y | (t1.y << 1) | (t2.y << 2);
}

struct BitTally {
    int flips = 0;   // flipped sites (both halves)
    int fdown = 0;   // flipped sites that were -1 (both halves)
    int u = 0;       // second half: unsatisfied bonds of the odd sites after the update
};

// Metropolis update of word g (32 sites of sublattice P) of one walker.
// Sw: the walker's bits [2][G]; JB: bond bits [2][6][G]; th_base: LDS byte
// address of the slot's threshold table (8 entries, entry e); smem: the work
// item's LDS; kb0/kb1: bits of k_s as all-zero/all-one masks for
// s = +1 / -1.
template <int L, int P>
__device__ __forceinline__ void bits_word(const SweepArgs &A, const SampleDev &d, uint32_t *Sw,
                                          const uint32_t *JB, const char *smem, uint32_t th_base, uint32_t g,
                                          uint32_t c1, uint32_t c2, const uint32_t kb0[3],
                                          const uint32_t kb1[3], BitTally &ty)
{
    using B = BitGeo<L>;
    constexpr int G = B::G, SEG = B::SEG, R = B::R, WPP = B::WPP;
    uint32_t *own = Sw + P * G;
    const uint32_t *oth = Sw + (1 - P) * G;
    const uint32_t z = g / WPP, y0 = R * (g % WPP);
    const uint32_t s = own[g], o = oth[g];
    uint32_t nyp, nym;
    if constexpr (R == L) {
        nyp = funnel(o, o, SEG);
        nym = funnel(o, o, 32 - SEG);
    } else {
        const uint32_t gyn = y0 + R < L ? g + 1 : g + 1 - WPP;
        const uint32_t gyp = y0 > 0 ? g - 1 : g - 1 + WPP;
        nyp = funnel(oth[gyn], o, SEG);
        nym = funnel(o, oth[gyp], 32 - SEG);
    }
    const uint32_t nzp = oth[g + WPP < G ? g + WPP : g + WPP - G];
    const uint32_t nzm = oth[g >= WPP ? g - WPP : g - WPP + G];
    const uint32_t up = sel(o >> 1, o << (SEG - 1), B::TOP);  // bit k <- bit k+1 of the row
    const uint32_t dn = sel(o << 1, o >> (SEG - 1), B::BOT);  // bit k <- bit k-1 of the row
    const uint32_t em = ((z + P) & 1) ? B::EVEN : ~B::EVEN;    // rows with eps = 1
    const uint32_t nxp = sel(o, up, em), nxm = sel(dn, o, em);
    const uint32_t *J = JB + P * 6 * G + g;
    const uint32_t u0 = xor3(s, nxp, J[0]), u1 = xor3(s, nxm, J[G]), u2 = xor3(s, nyp, J[2 * G]);
    const uint32_t u3 = xor3(s, nym, J[3 * G]), u4 = xor3(s, nzp, J[4 * G]), u5 = xor3(s, nzm, J[5 * G]);
    // c = u0 + ... + u5 per bit: two full adders, then the carry-save step
    const uint32_t a1 = xor3(u0, u1, u2), b1 = maj3(u0, u1, u2);
    const uint32_t a2 = xor3(u3, u4, u5), b2 = maj3(u3, u4, u5);
    const uint32_t C0 = a1 ^ a2, k = a1 & a2;
    const uint32_t C1 = xor3(b1, b2, k), C2 = maj3(b1, b2, k);
    // dE <= 0 iff c >= k_s: no borrow out of c - k_s
    const uint32_t K0 = sel(kb0[0], kb1[0], s), K1 = sel(kb0[1], kb1[1], s), K2 = sel(kb0[2], kb1[2], s);
    const uint32_t w0 = ~C0 & K0;
    const uint32_t w1 = (~C1 & K1) | (~C1 & w0) | (K1 & w0);
    const uint32_t w2 = (~C2 & K2) | (~C2 & w1) | (K2 & w1);
    const uint32_t D = ~w2;
    // class numbers e (c, or 7 - c for s = +1) as byte offsets 4 e, 8 sites per pair
    const uint32_t E0 = ~(C0 ^ s), E1 = ~(C1 ^ s), E2 = ~(C2 ^ s);
    uint32_t Q[8];
    const uint32_t sp = lds_addr(smem + SPREAD_OFF);
    spread3<0>(sp, E0, E1, E2, Q);
    spread3<1>(sp, E0, E1, E2, Q);
    spread3<2>(sp, E0, E1, E2, Q);
    spread3<3>(sp, E0, E1, E2, Q);
    // sites 31 .. 0, one Philox call per four (counter word 0 = 8 g + q); F
    // collects the accept bits (w < thr), each shifted in as the carry of F + F
    uint32_t F = 0;
#pragma unroll
    for (int q = 7; q >= 0; --q) {
        const u32x4 rw = philox4x32_10(8u * g + (uint32_t)q, c1, c2, d.sample_id, A.key0, A.key1);
        const uint32_t Qq = Q[q];
        F = shift_in_less(F, rw.w, lds_load(th_base + (Qq >> 24)));
        F = shift_in_less(F, rw.z, lds_load(th_base + ((Qq >> 16) & 0xFFu)));
        F = shift_in_less(F, rw.y, lds_load(th_base + ((Qq >> 8) & 0xFFu)));
        F = shift_in_less(F, rw.x, lds_load(th_base + (Qq & 0xFFu)));
    }
    F |= D;
    own[g] = s ^ F;
    ty.flips += __builtin_popcount(F);
    ty.fdown += __builtin_popcount(F & s);
    if constexpr (P == 1) {
        // after the update c' = 6 - c at flipped sites: sum c' = sum_k 2^k |C_k ^ F| - |F|
        ty.u += __builtin_popcount(C0 ^ F) + 2 * __builtin_popcount(C1 ^ F) + 4 * __builtin_popcount(C2 ^ F) -
                __builtin_popcount(F);
    }
}

__device__ __forceinline__ int lane_group_sum(int v, int width)
{
    for (int m = width >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

template <int L>
__device__ __forceinline__ void run_bits_item(const SweepArgs &A, const SampleDev &d, int r, char *smem)
{
    using B = BitGeo<L>;
    constexpr int N = B::N, G = B::G, SEG = B::SEG, R = B::R;
    const int nT = d.n_T, T = blockDim.x, tid = threadIdx.x;
    const BitsLdsOff o = bits_lds_offsets(L, nT);
    uint32_t *SB = (uint32_t *)(smem + o.spins);
    uint32_t *JB = (uint32_t *)(smem + o.J);
    uint32_t *TH = (uint32_t *)(smem + o.th);
    uint2 *SP = (uint2 *)(smem + o.spread);
    ItemLds I{};
    I.was = (int32_t *)(smem + o.was);
    I.sow = (int32_t *)(smem + o.sow);
    I.M = (int32_t *)(smem + o.M);
    I.dM = (int32_t *)(smem + o.dM);
    I.fl = (int32_t *)(smem + o.fl);
    I.sw = (int32_t *)(smem + o.sw);
    I.EJ = (long long *)(smem + o.EJ);
    I.dEJ = (long long *)(smem + o.dEJ);
    I.b64 = (double *)(smem + o.b64);

    const size_t sbase = (size_t)d.spin_off + (size_t)r * nT * N;
    const int gi = 2 * d.slot_off + r * nT;
    // spins: int8 [walker][parity][N/2] -> bits; word i covers bytes 32 i .. 32 i + 31
    for (int i = tid; i < nT * 2 * G; i += T) {
        const int4 *src = (const int4 *)(A.spins + sbase + (size_t)i * 32);
        const int4 v0 = src[0], v1 = src[1];
        SB[i] = pack4(v0.x) | pack4(v0.y) << 4 | pack4(v0.z) << 8 | pack4(v0.w) << 12 | pack4(v1.x) << 16 |
                pack4(v1.y) << 20 | pack4(v1.z) << 24 | pack4(v1.w) << 28;
    }
    block_copy(JB, A.Jbits + d.jb_off, (size_t)12 * G * 4);
    // k_s: smallest c with dE <= 0 for s = +1 (a = 1, b = 6 - c) and s = -1 (a = 0, b = c); 7 if none
    int k0 = 7, k1 = 7;
    for (int c = 6; c >= 0; --c) {
        if ((d.down_mask >> (7 + 6 - c)) & 1u) k0 = c;
        if ((d.down_mask >> c) & 1u) k1 = c;
    }
    for (int i = tid; i < nT * 8; i += T) {
        // entry e: s = -1 with c = e < k_-  (a = 0, b = c), or s = +1 with
        // c = 7 - e < k_+ (a = 1, b = 6 - c = e - 1); other entries are never used
        const int t = i >> 3, e = i & 7;
        const size_t row = ((size_t)d.slot_off + t) * 14;
        TH[i] = e < k1 ? A.lut[row + e] : (e >= 1 && 7 - e < k0) ? A.lut[row + 7 + e - 1] : 0u;
    }
    for (int v = tid; v < 256; v += T) {
        uint32_t lo = 0, hi = 0;
        for (int k = 0; k < 4; ++k) {
            lo |= ((v >> k) & 1u) * 4u << (8 * k);
            hi |= ((v >> (k + 4)) & 1u) * 4u << (8 * k);
        }
        SP[v] = make_uint2(lo, hi);
    }
    for (int i = tid; i < nT; i += T) {
        I.was[i] = A.was[gi + i];
        I.sow[A.was[gi + i]] = i;  // kept by exchange_pass from here on
        I.EJ[i] = A.EJ[gi + i];
        I.M[i] = A.M[gi + i];
        I.fl[i] = 0;
        I.sw[i] = 0;
        I.b64[i] = A.beta[d.slot_off + i];
    }
    uint32_t kb0[3], kb1[3];
    for (int i = 0; i < 3; ++i) {
        kb0[i] = ((k0 >> i) & 1) ? ~0u : 0u;
        kb1[i] = ((k1 >> i) & 1) ? ~0u : 0u;
    }
    __syncthreads();

    const int tpw = bits_tpw(L, nT);
    const int w = tid / tpw, lane = tid - w * tpw;
    const bool on = w < nT;
    uint32_t *Sw = SB + (size_t)(on ? w : 0) * 2 * G;
    const double hd = (double)d.h32;
    const int64_t n0 = A.state[0];
    int64_t next_meas = next_measurement(n0, A.measure_every, A.measure_start);
    int64_t f = 0;  // frame of the next measurement within this chunk
    for (int it = 0; it < A.K; ++it) {
        const int64_t n = n0 + it;
        const int t = on ? I.sow[w] : 0;
        const uint32_t th_base = lds_addr(smem + TH_OFF + 32 * t);
        const uint32_t c2 = (PURPOSE_METROPOLIS << 28) | ((uint32_t)t << 1) | (uint32_t)r;
        BitTally ty;
        if (on) {
            const uint32_t c1 = (uint32_t)(2 * n);
#pragma unroll 1
            for (uint32_t g = lane; g < G; g += tpw) bits_word<L, 0>(A, d, Sw, JB, smem, th_base, g, c1, c2, kb0, kb1, ty);
        }
        __syncthreads();
        if (on) {
            const uint32_t c1 = (uint32_t)(2 * n + 1);
#pragma unroll 1
            for (uint32_t g = lane; g < G; g += tpw) bits_word<L, 1>(A, d, Sw, JB, smem, th_base, g, c1, c2, kb0, kb1, ty);
            const int sf = lane_group_sum(ty.flips, tpw), sd = lane_group_sum(ty.fdown, tpw);
            const int su = lane_group_sum(ty.u, tpw);
            if (lane == 0) {
                // every bond has one odd end: E_J = (unsatisfied) - (satisfied) = 2 U - 3 N
                I.EJ[w] = 2 * (long long)su - 3 * (long long)N;
                I.M[w] += -2 * (sf - 2 * sd);
                I.fl[t] += sf;
            }
        }
        __syncthreads();
        exchange_pass(A, d, r, n, I, 1.0, hd);
        __syncthreads();
        // Snapshot for the overlap measurement, in slot order: row (y, z) of
        // L bits interleaves the two sublattices' rows.
        const int64_t done = n + 1;
        if (done == next_meas) {
            next_meas += A.measure_every;
            uint32_t *dst = A.frames + f * A.frame_words + d.frame_off + (size_t)r * nT * L * L;
            for (int i = tid; i < nT * L * L; i += T) {
                const int ts = i / (L * L), row = i - ts * (L * L);
                const int y = row % L, zz = row / L;
                const int g = row / R, sh = (row % R) * SEG;
                const uint32_t *Wb = SB + (size_t)I.was[ts] * 2 * G;
                const int pe = (y + zz) & 1;  // sublattice on the even x positions
                const uint32_t ev = (Wb[pe * G + g] >> sh) & ((1u << SEG) - 1u);
                const uint32_t od = (Wb[(1 - pe) * G + g] >> sh) & ((1u << SEG) - 1u);
                dst[i] = spread2(ev) | (spread2(od) << 1);
            }
            for (int ts = tid; ts < nT; ts += T) {
                const int ww = I.was[ts];
                A.frameE[f * 2 * A.total_slots + gi + ts] = (double)I.EJ[ww] - hd * (double)I.M[ww];
            }
            ++f;
            __syncthreads();  // the next sweep changes the spins read here
        }
    }
    __syncthreads();
    for (int i = tid; i < nT * 2 * G; i += T) {
        const uint32_t b = SB[i];
        int4 *dst = (int4 *)(A.spins + sbase + (size_t)i * 32);
        dst[0] = make_int4((int)unpack4(b & 15u), (int)unpack4((b >> 4) & 15u), (int)unpack4((b >> 8) & 15u),
                           (int)unpack4((b >> 12) & 15u));
        dst[1] = make_int4((int)unpack4((b >> 16) & 15u), (int)unpack4((b >> 20) & 15u),
                           (int)unpack4((b >> 24) & 15u), (int)unpack4(b >> 28));
    }
    for (int i = tid; i < nT; i += T) {
        A.was[gi + i] = I.was[i];
        A.EJ[gi + i] = I.EJ[i];
        A.M[gi + i] = I.M[i];
        A.flips[gi + i] += I.fl[i];
        A.swaps[gi + i] += I.sw[i];
    }
    __syncthreads();
}

// VAR only separates the symbol of the one-sample-per-launch comparator.
template <int L, int VAR>
__global__ void __launch_bounds__(1024) bits_sweep_kernel(SweepArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (int item = blockIdx.x; item < A.n_items; item += gridDim.x) {
        const int code = A.items[item];
        run_bits_item<L>(A, A.samples[code >> 1], code & 1, smem);
    }
}

template __global__ void bits_sweep_kernel<8, 0>(SweepArgs);
template __global__ void bits_sweep_kernel<8, 1>(SweepArgs);
template __global__ void bits_sweep_kernel<16, 0>(SweepArgs);
template __global__ void bits_sweep_kernel<16, 1>(SweepArgs);
template __global__ void bits_sweep_kernel<32, 0>(SweepArgs);
template __global__ void bits_sweep_kernel<32, 1>(SweepArgs);

}  // namespace ea
