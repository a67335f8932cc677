// ea_item.hpp -- device helpers shared by the LDS-resident engines: block
// copies, wave and lane-group sums, the LDS frame of one (sample, chain) work
// item and the replica-exchange pass over it.
#pragma once

#include "ea_device.hpp"
#include "ea_types.hpp"

namespace ea {

// The threads that run one work item: the whole workgroup, or one of the
// equal, wave-aligned teams a batch workgroup is split into (each team with
// its own LDS region; every team passes the same barriers).  A ghost team
// computes like a real one on a copy of a real item but writes nothing to
// global memory (it fills a batch unit that has fewer items than teams).
struct Team {
    int tid;     // thread index within the team
    int T;       // threads in the team
    bool ghost;
};

__device__ __forceinline__ Team whole_block() { return Team{(int)threadIdx.x, (int)blockDim.x, false}; }

// Team-cooperative byte copy, 16 bytes at a time when both ends allow it;
// four copies in flight per thread.
__device__ __forceinline__ void block_copy(void *__restrict__ dst, const void *__restrict__ src, size_t bytes,
                                           const Team tm = whole_block())
{
    const int T = tm.T, tid = tm.tid;
    if ((((uintptr_t)dst | (uintptr_t)src | bytes) & 15) == 0) {
        int4 *__restrict__ d = (int4 *)dst;
        const int4 *__restrict__ s = (const int4 *)src;
        const size_t n = bytes / 16;
        size_t i = tid;
        for (; i + 3 * (size_t)T < n; i += 4 * (size_t)T) {
            const int4 a = s[i], b = s[i + T], c = s[i + 2 * T], e = s[i + 3 * T];
            d[i] = a;
            d[i + T] = b;
            d[i + 2 * T] = c;
            d[i + 3 * T] = e;
        }
        for (; i < n; i += T) d[i] = s[i];
    } else {
        int8_t *d = (int8_t *)dst;
        const int8_t *s = (const int8_t *)src;
        for (size_t i = tid; i < bytes; i += T) d[i] = s[i];
    }
}

// count walkers of bytes each (a multiple of 8) from consecutive blocks at
// glob to blocks lstride bytes apart at lds (to_lds), or back, in 8-byte words.
__device__ __forceinline__ void copy_walkers(int8_t *lds, size_t lstride, int8_t *glob, int count, size_t bytes,
                                             bool to_lds, const Team tm = whole_block())
{
    const int T = tm.T, tid = tm.tid;
    const size_t per = bytes / 8, total = per * (size_t)count;
    for (size_t i = tid; i < total; i += T) {
        const size_t w = i / per, j = i - w * per;
        uint2 *l = (uint2 *)(lds + w * lstride) + j;
        uint2 *g = (uint2 *)(glob + w * bytes) + j;
        if (to_lds) *l = *g;
        else *g = *l;
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

// Pointers into the dynamic LDS of one work item.
struct ItemLds {
    int8_t *S;
    void *J;
    int32_t *was, *sow, *M, *dM, *fl, *sw;
    long long *EJ, *dEJ;
    uint32_t *lut;
    float *b32;
    double *b64;
};

// The descriptor of a workgroup's sample, read into scalar registers: the
// item code is the same for every lane, and descriptors are read-only during a
// launch, so the read may go through the scalar cache.
__device__ __forceinline__ SampleDev sample_of_item(const SampleDev *samples, int idx)
{
    typedef const __attribute__((address_space(4))) uint32_t *ConstWords;
    static_assert(sizeof(SampleDev) % 4 == 0, "descriptor is read in 32-bit words");
    const ConstWords src = (ConstWords)(samples + __builtin_amdgcn_readfirstlane(idx));
    uint32_t w[sizeof(SampleDev) / 4];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(SampleDev) / 4); ++k) w[k] = src[k];
    SampleDev d;
    __builtin_memcpy(&d, w, sizeof d);
    return d;
}

__device__ __forceinline__ ItemLds item_lds(char *smem, int L, int nT, int jkind)
{
    const LdsOff o = lds_offsets(L, nT, jkind);
    ItemLds p;
    p.S = (int8_t *)(smem + o.spins);
    p.J = (void *)(smem + o.J);
    p.was = (int32_t *)(smem + o.was);
    p.sow = (int32_t *)(smem + o.sow);
    p.M = (int32_t *)(smem + o.M);
    p.dM = (int32_t *)(smem + o.dM);
    p.fl = (int32_t *)(smem + o.fl);
    p.sw = (int32_t *)(smem + o.sw);
    p.EJ = (long long *)(smem + o.EJ);
    p.dEJ = (long long *)(smem + o.dEJ);
    p.lut = (uint32_t *)(smem + o.lut);
    p.b32 = (float *)(smem + o.b32);
    p.b64 = (double *)(smem + o.b64);
    return p;
}

// Replica exchange of neighbouring slots (t, t+1), t = n&1, n&1 + 2, ...
// (Methods: parallel tempering; even-odd pairs alternate with the sweep
// parity).  D = (beta_t - beta_{t+1}) (E_t - E_{t+1}) in binary64, E_w =
// energy(w); accepted iff D >= 0 or u53 < exp_ea64(D) (decided by
// exchange_accept), u53 from the exchange counter (0, n, (1 << 28) | (t << 1)
// | r, sample).  Swaps walker labels only, in both maps (was: slot -> walker,
// sow: walker -> slot), so the sweep that follows reads its temperatures
// without rebuilding sow.
template <class Energy>
__device__ __forceinline__ void exchange_pass_e(const SweepArgs &A, const SampleDev &d, int r, int64_t n,
                                                const ItemLds &I, Energy energy, const Team tm)
{
    const int nT = d.n_T, T = tm.T;
    for (int j = tm.tid;; j += T) {
        const int t = (int)(n & 1) + 2 * j;
        if (t + 1 >= nT) break;
        const int w0 = I.was[t], w1 = I.was[t + 1];
        const double D = (I.b64[t] - I.b64[t + 1]) * (energy(w0) - energy(w1));
        bool acc = D >= 0.0;
        if (!acc) {
            const u32x4 q = philox4x32_10(0u, (uint32_t)n,
                                          (PURPOSE_EXCHANGE << 28) | ((uint32_t)t << 1) | (uint32_t)r,
                                          d.sample_id, A.key0, A.key1);
            acc = exchange_accept(u53_of(q.x, q.y), D);
        }
        if (acc) {
            I.was[t] = w1;
            I.was[t + 1] = w0;
            I.sow[w1] = t;
            I.sow[w0] = t + 1;
            I.sw[t] += 1;
        }
    }
}

// The same with E_w = EJ_w unit - h M_w from the walker arrays.
__device__ __forceinline__ void exchange_pass(const SweepArgs &A, const SampleDev &d, int r, int64_t n,
                                              const ItemLds &I, double unit, double hd, const Team tm = whole_block())
{
    exchange_pass_e(
        A, d, r, n, I, [&](int w) { return (double)I.EJ[w] * unit - hd * (double)I.M[w]; }, tm);
}

// v of the lane K places along in the same row of 16 lanes (rotation).
template <int K>
__device__ __forceinline__ int row_rotate(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x120 + K, 0xF, 0xF, true);
}

template <int K>
__device__ __forceinline__ long long row_rotate(long long v)
{
    // (the halves as a register pair: assembled with shifts and ors, the
    // compiler adds the halves into a sum one at a time)
    typedef int int2v __attribute__((ext_vector_type(2)));
    int2v h = __builtin_bit_cast(int2v, v);
    h.x = row_rotate<K>(h.x);
    h.y = row_rotate<K>(h.y);
    return __builtin_bit_cast(long long, h);
}

// v of lane (this lane XOR K) within its aligned group of four (K = 1 or 2).
template <int K>
__device__ __forceinline__ int quad_xor(int v)
{
    static_assert(K == 1 || K == 2, "quad permutation");
    return __builtin_amdgcn_mov_dpp(v, K == 1 ? 0xB1 : 0x4E, 0xF, 0xF, true);
}

template <int K>
__device__ __forceinline__ long long quad_xor(long long v)
{
    typedef int int2v __attribute__((ext_vector_type(2)));
    int2v h = __builtin_bit_cast(int2v, v);
    h.x = quad_xor<K>(h.x);
    h.y = quad_xor<K>(h.y);
    return __builtin_bit_cast(long long, h);
}

// Sum over aligned groups of W = 4 or 16 consecutive lanes, every lane of the
// group active (DPP: permutations within four lanes, rotations within a row).
template <int W, class V>
__device__ __forceinline__ V group_sum_dpp(V v)
{
    static_assert(W == 4 || W == 16, "group of four lanes or a row");
    if constexpr (W == 4) {
        v += quad_xor<1>(v);
        v += quad_xor<2>(v);
    } else {
        v += row_rotate<8>(v);
        v += row_rotate<4>(v);
        v += row_rotate<2>(v);
        v += row_rotate<1>(v);
    }
    return v;
}

// Sum of v over the lanes of this lane's row of 16 whose index agrees with
// this lane's modulo S (S = 1, 2, 4, 8 or 16, uniform): rotations by S, 2S,
// .., 8.  Every lane of the wave must be active.
template <class V>
__device__ __forceinline__ V row_residue_sum(V v, int S)
{
    if (S <= 1) v += row_rotate<1>(v);
    if (S <= 2) v += row_rotate<2>(v);
    if (S <= 4) v += row_rotate<4>(v);
    if (S <= 8) v += row_rotate<8>(v);
    return v;
}

}  // namespace ea
