// ea_update.hpp -- the Metropolis update of one int8x4 word with Gaussian
// couplings, shared by the row, HBM and group engines, and the energy tallies
// taken from its result.
#pragma once

#include "ea_device.hpp"

namespace ea {

// f with its sign flipped iff byte i of m is 0x80: one SDWA xor of that byte
// into the sign byte of f (the other bytes of f are kept).
__device__ __forceinline__ float flip_by_byte(float f, uint32_t m, int i)
{
    switch (i) {
    case 0:
        asm("v_xor_b32_sdwa %0, %1, %0 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_0 src1_sel:BYTE_3"
            : "+v"(f) : "v"(m));
        break;
    case 1:
        asm("v_xor_b32_sdwa %0, %1, %0 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_1 src1_sel:BYTE_3"
            : "+v"(f) : "v"(m));
        break;
    case 2:
        asm("v_xor_b32_sdwa %0, %1, %0 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_2 src1_sel:BYTE_3"
            : "+v"(f) : "v"(m));
        break;
    default:
        asm("v_xor_b32_sdwa %0, %1, %0 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_3 src1_sel:BYTE_3"
            : "+v"(f) : "v"(m));
        break;
    }
    return f;
}

// Metropolis update of one int8x4 word Sv: four spins (bytes +-1), each with
// its six neighbour spins in bytes of the same position of Xa, Xs, Yp, Ym, Zp,
// Zm and its six bonds (int32 multiples of 2^-18) in Ja[i] .. Jzn[i].  The four
// bytes are four sites of one walker (row and HBM engines) or one site of four
// walkers (group engine).  rw holds byte i's Philox word in word i; b2_of(i)
// returns 2 beta32 of byte i's slot (read only on the exact path).  Returns
// the flip mask (0xFE in the bytes of accepted sites) and the integer local
// field of every byte in Sus: S_u (S_J = S_u 2^-18), or with FOLD S_u + hgrid.
//
// Decision: with f = fl32(S_J + h) and g = -s_i f (exact), x = -fl32(beta32 dE)
// is fl32(2 beta32 g) (the same real number, rounded once), dE <= 0 iff x >= 0,
// exp_ea32 is 0 below -86.  The random word is decided by the sign of the gap
// fl32(W - 2^(y + 32)) when its magnitude exceeds M (accept_gap), otherwise by
// x >= 0 or U 2^-24 < exp_ea32(x), the contract's rule; one wave-uniform
// branch per word takes that test for all four bytes in every lane as soon as
// one byte of one lane needs it.  The exponent y estimates x log2(e):
//   FOLD = false: y = fl32(c' g), ka[i] = c' = two_beta_log2e(beta32);
//   FOLD = true:  y = -s_i fl32(fl32(S_u + hgrid) ka[i] + kb[i]) with
//     ka[i] = c' 2^-18 and kb[i] = fl32(c' (h - hgrid 2^-18)), one fused
//     operation for the field and the temperature together.
// ea_verify_exp_bracket proves both signs of the gap safe for every binary32 x
// and every y the two forms can produce (within a relative 2^-21 of x log2(e)
// plus 2^-20; the bound on the second form needs beta32 <= 2^20).
template <bool FOLD, class B2>
__device__ __forceinline__ uint32_t update_word_gauss(uint32_t Sv, uint32_t Xa, uint32_t Xs, uint32_t Yp,
                                                      uint32_t Ym, uint32_t Zp, uint32_t Zm, const int Ja[4],
                                                      const int Js[4], const int Jy[4], const int Jyn[4],
                                                      const int Jz[4], const int Jzn[4], const u32x4 rw,
                                                      const float ka[4], const float kb[4], B2 b2_of, float h32,
                                                      int hgrid, int Sus[4])
{
    const uint32_t words[4] = {rw.x, rw.y, rw.z, rw.w};
    const uint32_t up = ~Sv & 0x80808080u;  // 0x80 in the bytes with s_i = +1
    float gap[4];
    float gmin = __builtin_inff();  // the least |gap| of the four bytes
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int sh = 8 * i;
        int Su = __mul24(__builtin_amdgcn_sbfe((int)Xa, sh, 8), Ja[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Xs, sh, 8), Js[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Yp, sh, 8), Jy[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Ym, sh, 8), Jyn[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Zp, sh, 8), Jz[i]);
        Su += __mul24(__builtin_amdgcn_sbfe((int)Zm, sh, 8), Jzn[i]);
        if constexpr (FOLD) Su += hgrid;
        Sus[i] = Su;
        float y;
        if constexpr (FOLD) {
            y = flip_by_byte(__builtin_fmaf((float)Su, ka[i], kb[i]), up, i);
        } else {
            // f = fl32(S_J + h): S_J = Su 2^-18 exactly, so the fused form rounds once, as the sum does
            y = ka[i] * flip_by_byte(__builtin_fmaf((float)Su, 0x1p-18f, h32), up, i);  // c' (-s_i f)
        }
        gap[i] = accept_gap(y, (float)words[i]);
        gmin = __builtin_fminf(gmin, __builtin_fabsf(gap[i]));
    }
    // With every |gap| above M a byte is accepted iff its gap is negative:
    // byte permutes with selectors 9 and 11 replicate the sign bit of the low
    // and high source word into a whole byte.
    uint32_t fm = (__builtin_amdgcn_perm(__float_as_uint(gap[1]), __float_as_uint(gap[0]), 0x0C0C0B09u) |
                   __builtin_amdgcn_perm(__float_as_uint(gap[3]), __float_as_uint(gap[2]), 0x0B090C0Cu)) &
                  0xFEFEFEFEu;
    // If any lane of the wave has a byte with |gap| <= M, every lane takes the
    // exact test for all four bytes, which the gap only anticipates.  One
    // wave-uniform branch per word lets the four bytes' chains interleave.
    if (__builtin_amdgcn_ballot_w64(gmin <= ACCEPT_MARGIN) != 0) {
        fm = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // S_u taken back from the stored sum here only (the empty asm keeps
            // the compiler from holding the sum without hgrid for this path,
            // which would cost the main path a separate add)
            int su = Sus[i];
            asm volatile("" : "+v"(su));
            if constexpr (FOLD) su -= hgrid;
            const float g = flip_by_byte(__builtin_fmaf((float)su, 0x1p-18f, h32), up, i);  // -s_i f
            const float x = b2_of(i) * g;                                                  // = -fl32(beta dE)
            const bool accept = x >= 0.0f || (float)(words[i] >> 8) * 0x1p-24f < exp_ea32(x);
            fm |= accept ? 0xFEu << (8 * i) : 0u;
        }
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
