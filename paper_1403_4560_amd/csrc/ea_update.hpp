// ea_update.hpp -- the Metropolis update of one int8x4 word with Gaussian
// couplings, shared by the row, HBM and group engines, and the energy tallies
// taken from its result.
#pragma once

#include "ea_device.hpp"

namespace ea {

// Metropolis update of one int8x4 word Sv: four spins (bytes +-1), each with
// its six neighbour spins in bytes of the same position of Xa, Xs, Yp, Ym, Zp,
// Zm and its six bonds (int32 multiples of 2^-18) in Ja[i] .. Jzn[i].  The four
// bytes are four sites of one walker (row and HBM engines) or one site of four
// walkers (group engine).  rw holds byte i's Philox word in word i; m2b[i] =
// -2 beta32 of byte i's slot.  Returns the flip mask (0xFE in the bytes of
// accepted sites) and S_u of every byte in Sus (S_J = S_u 2^-18).
//
// Decision: x = -fl32(beta32 dE) is formed as fl32((-2 beta32 s_i) f) (the same
// real number, rounded once), dE <= 0 iff x >= 0, exp_ea32 is 0 below -86.  The
// random word is decided by accept_bracket when it falls outside the bracket
// (ea_verify_exp_bracket proves the bracket safe for every x <= 0, and that
// below -86 no word falls under it), otherwise by U 2^-24 < exp_ea32(x)
// itself.  For x >= 0 both routes accept, as the contract's dE <= 0 rule does.
__device__ __forceinline__ uint32_t update_word_gauss(uint32_t Sv, uint32_t Xa, uint32_t Xs, uint32_t Yp,
                                                      uint32_t Ym, uint32_t Zp, uint32_t Zm, const int Ja[4],
                                                      const int Js[4], const int Jy[4], const int Jyn[4],
                                                      const int Jz[4], const int Jzn[4], const u32x4 rw,
                                                      const float m2b[4], float h32, int Sus[4])
{
    const uint32_t words[4] = {rw.x, rw.y, rw.z, rw.w};
    const uint32_t nS = ~Sv;  // byte sign bit set iff s_i = +1
    uint32_t fm = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int sh = 8 * i;
        int Su = __mul24(__builtin_amdgcn_sbfe((int)Xa, sh, 8), Ja[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Xs, sh, 8), Js[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Yp, sh, 8), Jy[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Ym, sh, 8), Jyn[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Zp, sh, 8), Jz[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Zm, sh, 8), Jzn[i]);
        Sus[i] = Su;
        // f = fl32(S_J + h): S_J = Su 2^-18 exactly, so the fused form rounds once, as the sum does
        const float f = __builtin_fmaf((float)Su, 0x1p-18f, h32);
        // c = -2 beta32 s_i: the sign bit of 2 beta32 set iff s_i = +1 (exact)
        const uint32_t b2 = __float_as_uint(m2b[i]) & 0x7FFFFFFFu;  // 2 beta32
        const float c = __uint_as_float(__builtin_amdgcn_ubfe(nS, sh + 7, 1) << 31 | b2);
        const float x = c * f;                         // = -fl32(beta * dE)
        float lo, hi;
        accept_bracket(x, lo, hi);
        const float Wf = (float)words[i];
        const bool below = Wf < lo, under_hi = Wf < hi;  // lo < hi, so below implies under_hi
        bool accept = below;
        // If a lane of the wave has lo <= W < hi (the two lane masks differ),
        // every lane takes the exact test, which the bracket only anticipates.
        if (__builtin_amdgcn_ballot_w64(under_hi) != __builtin_amdgcn_ballot_w64(below))
            accept = (float)(words[i] >> 8) * 0x1p-24f < exp_ea32(x);
        fm |= accept ? 0xFEu << sh : 0u;
    }
    return fm;
}

// Sum over accepted bytes of (S_u XOR m), m = 0 for s_i = +1 and -1 for
// s_i = -1: the sum of s_i S_u over accepted sites is this plus the number of
// accepted down spins.
__device__ __forceinline__ int tally_delta(uint32_t Sv, uint32_t fm, const int Sus[4])
{
    int a = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if ((fm >> (8 * i)) & 0xFFu) a += Sus[i] ^ __builtin_amdgcn_sbfe((int)Sv, 8 * i + 7, 1);
    return a;
}

// After the update: accE += (S_u XOR m') over all four bytes and nd += the
// number of -1 spins, m' from the updated spin, so that accE + nd is the sum of
// s_i' S_u with the updated spins.  On the second half-sweep that sum over a
// walker's odd sites is minus its whole coupling energy: every bond joins one
// even and one odd site, and the even spins no longer change.  S_u can reach
// 6 (2^21 - 1) in magnitude, beyond a 24-bit multiplier, so the sign is
// applied by XOR.
__device__ __forceinline__ void tally_final(uint32_t Sv, uint32_t fm, const int Sus[4], int &accE, int &nd)
{
    const uint32_t Sn = Sv ^ fm;
#pragma unroll
    for (int i = 0; i < 4; ++i) accE += Sus[i] ^ __builtin_amdgcn_sbfe((int)Sn, 8 * i + 7, 1);
    nd += __builtin_popcount(Sn & 0x80808080u);
}

// The same per byte (group engine: byte i is walker i of the word's quad).
__device__ __forceinline__ void tally_final_lanes(uint32_t Sv, uint32_t fm, const int Sus[4], int accE[4],
                                                  int nd[4])
{
    const uint32_t Sn = Sv ^ fm;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = __builtin_amdgcn_sbfe((int)Sn, 8 * i + 7, 1);
        accE[i] += Sus[i] ^ m;
        nd[i] -= m;
    }
}

}  // namespace ea
