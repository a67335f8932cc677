// ea_device.hpp -- device primitives of the gfx950 engine: counter-based
// random numbers and the in-house exponentials of the acceptance tests.
//
// Compiled with -ffp-contract=off: every floating-point operation below is one
// IEEE operation rounded to nearest even, so the results are reproducible bit
// for bit by any conforming implementation of the same steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ea {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
// as 1, 2, 3", SC'11).  Each of the ten rounds forms the 64-bit products of
// counter words 0 and 2 with the two round multipliers; the new counter is
// (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1, lo(c0*M0)).  The key
// advances by the Weyl increments between rounds.
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // truth table of a ^ b ^ c
}

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0, n2;
        if (round < 2) {
            // plain xors: in the first two rounds one side of each product is
            // often loop-invariant, and the compiler can then hoist part of it
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
            n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += W0;
        k1 += W1;
    }
    return {c0, c1, c2, c3};
}

// Counter purposes (bits 28..31 of counter word 2).
constexpr uint32_t PURPOSE_METROPOLIS = 0u;
constexpr uint32_t PURPOSE_EXCHANGE = 1u;

// e^x for -86 <= x <= 0 in binary32: Cody-Waite reduction x = k ln2 + r with
// the split ln2 = C1 + C2 (C1 keeps 16 significant bits so k*C1 is exact for
// |k| <= 255), then the degree-7 Taylor polynomial of e^r in Horner form and
// an exact scaling by 2^k.  x < -86 gives 0.  Constants (IEEE binary32 bit
// patterns): 1/ln2, ln2 rounded then its 8 low bits cleared, the rounded
// remainder ln2 - C1, and the rounded reciprocal factorials 1/j!.
__device__ __forceinline__ float exp_ea32(float x)
{
    const float LOG2E = __uint_as_float(0x3FB8AA3Bu);
    const float C1 = __uint_as_float(0x3F317200u);
    const float C2 = __uint_as_float(0x35BFBE8Eu);
    const float xc = fmaxf(x, -100.0f);  // keeps k in range; result masked below
    const float k = __builtin_rintf(xc * LOG2E);
    const float r = (xc - k * C1) - k * C2;
    float p = __uint_as_float(0x39500D01u);          // 1/7!
    p = p * r + __uint_as_float(0x3AB60B61u);        // 1/6!
    p = p * r + __uint_as_float(0x3C088889u);        // 1/5!
    p = p * r + __uint_as_float(0x3D2AAAABu);        // 1/4!
    p = p * r + __uint_as_float(0x3E2AAAABu);        // 1/3!
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    const float v = __builtin_amdgcn_ldexpf(p, (int)k);
    return x < -86.0f ? 0.0f : v;
}

// e^x for -700 <= x <= 0 in binary64, the same construction: C1 keeps 42
// significant bits (11 low bits of fl64(ln2) cleared), degree-13 Taylor
// polynomial with rounded 1/j!, x < -700 gives 0.
__device__ __forceinline__ double exp_ea64(double x)
{
    const double LOG2E = __longlong_as_double(0x3FF71547652B82FEll);
    const double C1 = __longlong_as_double(0x3FE62E42FEFA3800ll);
    const double C2 = __longlong_as_double(0x3D2EF35793C76730ll);
    const double xc = fmax(x, -800.0);
    const double k = __builtin_rint(xc * LOG2E);
    const double r = (xc - k * C1) - k * C2;
    double p = __longlong_as_double(0x3DE6124613A86D09ll);        // 1/13!
    p = p * r + __longlong_as_double(0x3E21EED8EFF8D898ll);       // 1/12!
    p = p * r + __longlong_as_double(0x3E5AE64567F544E4ll);       // 1/11!
    p = p * r + __longlong_as_double(0x3E927E4FB7789F5Cll);       // 1/10!
    p = p * r + __longlong_as_double(0x3EC71DE3A556C734ll);       // 1/9!
    p = p * r + __longlong_as_double(0x3EFA01A01A01A01All);       // 1/8!
    p = p * r + __longlong_as_double(0x3F2A01A01A01A01All);       // 1/7!
    p = p * r + __longlong_as_double(0x3F56C16C16C16C17ll);       // 1/6!
    p = p * r + __longlong_as_double(0x3F81111111111111ll);       // 1/5!
    p = p * r + __longlong_as_double(0x3FA5555555555555ll);       // 1/4!
    p = p * r + __longlong_as_double(0x3FC5555555555555ll);       // 1/3!
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    const double v = __builtin_amdgcn_ldexp(p, (int)k);
    return x < -700.0 ? 0.0 : v;
}

// Acceptance gap.  The engines form an exponent y that estimates x log2(e),
// x = -fl32(beta32 dE), from the per-slot constant c' = fl32(2 beta32 log2 e)
// (update_word_gauss gives the two forms and their rounding bound), and the
// hardware estimate a = 2^y of exp_ea32(x).  With W = fl32(w) for the 32-bit
// random word w (so |W - w| <= 128), U = w >> 8 the 24-bit uniform numerator,
// A = a 2^32,
// T = exp_ea32(x) 2^32 and the gap g = fl32(W - A) (one fused rounding):
//   g < -M  =>  W - A < -M  =>  U <= w/256 < (A - M + 128)/256,
//   g >  M  =>  W - A >  M  =>  U >  w/256 - 1 > (A + M - 384)/256,
// so T - (M - 384) <= A <= T + (M - 128) makes g < -M a correct accept and
// g > M a correct reject.  ea_verify_exp_bracket checks, for every binary32 x,
// that pair of inequalities (T = 0 below -86; for x > 0, where the exact test
// accepts, only A >= 2^32 - M + 384, so that g > M cannot happen) at both ends
// of the range of a over every y within a relative 2^-21 of x log2(e) plus
// 2^-20, using that the hardware exponential is monotone (checked on every
// binary32 input by the same call).  Inside [-M, M] the exact test decides.
constexpr float ACCEPT_MARGIN = 8192.0f;  // M

// c' of a slot: fl32(2 beta32 log2 e), one rounding (2 beta32 is exact).
__device__ __forceinline__ float two_beta_log2e(float b32) { return (2.0f * b32) * __uint_as_float(0x3FB8AA3Bu); }

__device__ __forceinline__ float accept_gap(float y, float W)
{
    return __builtin_fmaf(__builtin_amdgcn_exp2f(y), -0x1p32f, W);
}

// 24-bit and 53-bit uniforms in [0, 1) from Philox output words.
__device__ __forceinline__ float u24_of(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ double u53_of(uint32_t w0, uint32_t w1)
{
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * 0x1p-53;
}

// Replica-exchange test for D < 0: returns u < exp_ea64(D), u a 53-bit
// uniform (a multiple of 2^-53 in [0, 1)), deciding from the hardware
// exponential wherever that is safe.
//   D < -40: exp_ea64(D) < e^-40 (1 + 2^-50) < 2^-57 < 2^-53 <= u unless u = 0.
//   -40 <= D < 0: e = 2^y, y = fl32(D log2 e) with |t| < 58 for t = D log2 e,
//     so |y - t| <= 2^-19 (half an ulp at |t| < 64); the hardware exp2 is
//     within a relative 2^-22 of 2^y on y in [-58, 0] (checked on every
//     binary32 there by ea_verify_exchange_bracket), and exp_ea64 within 2^-50
//     of e^D.  So e / exp_ea64(D) lies within 1 +- 1.7e-6, well inside the
//     margin 2^-16 = 1.5e-5: u < e (1 - 2^-16) implies u < exp_ea64(D), and
//     u > e (1 + 2^-16) implies u > exp_ea64(D).  Between the two (about 3e-5
//     of the draws), and for u = 0, exp_ea64 decides.
constexpr double EXCHANGE_FAST_MIN = -40.0;
constexpr double EXCHANGE_MARGIN = 0x1p-16;

__device__ __forceinline__ bool exchange_accept(double u, double D)
{
    if (u != 0.0) {
        if (D < EXCHANGE_FAST_MIN) return false;
        const float y = (float)(D * __longlong_as_double(0x3FF71547652B82FEll));  // D log2(e)
        const double e = (double)__builtin_amdgcn_exp2f(y);
        if (u < e * (1.0 - EXCHANGE_MARGIN)) return true;
        if (u > e * (1.0 + EXCHANGE_MARGIN)) return false;
    }
    return u < exp_ea64(D);
}

}  // namespace ea
