// ea_exact.hpp -- exact sums of binary64 values, rounded once.
//
// The disorder average of eqs. 3-6 (the overline: an average over the
// realizations of one model at one field and one temperature ladder) is taken
// as the exact sum of the per-sample thermal means rounded once to binary64
// (nearest, ties to even) and then divided by the sample count; a
// leave-one-sample-out replicate of the jackknife (Methods, last paragraph) is
// the exact sum of the other samples' values, rounded once, divided by the
// count less one.  No result then depends on the order in which threads or
// atomics visit the samples.
//
// Representation.  Every finite binary64 is an integer multiple of 2^-1074.
// An exact sum is XL signed 64-bit limbs, limb k weighing 2^(32k) such units.
// A value adds its 53-bit significand, cut into three 32-bit digits, to three
// consecutive limbs, so each limb grows by less than 2^32 per value: fewer
// than 2^30 values can never overflow a limb, and the additions commute (plain
// integer adds, or integer atomics in LDS).  Normalizing carries every limb
// into [0, 2^32) and leaves the sign as a final carry of 0 or -1.  Non-finite
// values are counted apart (NaN, +inf, -inf) and decide the result as IEEE
// addition would: any NaN, or +inf together with -inf, gives NaN; otherwise an
// infinity wins.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ea {

// Limbs: bit offsets 0 .. 2097 hold one value (significand at offset up to
// 2045, 53 bits); the rest is headroom for the carries of up to 2^30 values.
constexpr int XL = 68;

struct ExactDigits {
    int i;               // lowest limb touched
    int64_t d0, d1, d2;  // signed digits for limbs i, i+1, i+2
};

// The three digits of a finite x (negated when neg).  x = 0 gives zeros.
__device__ __forceinline__ ExactDigits exact_digits(double x, bool neg)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const int be = (int)((b >> 52) & 0x7ff);
    const uint64_t frac = b & ((1ull << 52) - 1);
    const uint64_t m = be ? (frac | (1ull << 52)) : frac;  // x = m 2^(o - 1074)
    const int o = be ? be - 1 : 0;
    const int sh = o & 31;
    const uint64_t lo = m << sh;                       // bits 0..63 of m 2^sh
    const uint64_t hi = sh ? (m >> (64 - sh)) : 0ull;  // bits 64..84
    ExactDigits r;
    r.i = o >> 5;
    r.d0 = (int64_t)(lo & 0xffffffffull);
    r.d1 = (int64_t)(lo >> 32);
    r.d2 = (int64_t)hi;
    if (neg != ((b >> 63) != 0)) {
        r.d0 = -r.d0;
        r.d1 = -r.d1;
        r.d2 = -r.d2;
    }
    return r;
}

// lim += x (or -= x), x finite.
__device__ __forceinline__ void exact_add(int64_t *lim, double x, bool neg = false)
{
    const ExactDigits g = exact_digits(x, neg);
    lim[g.i] += g.d0;
    lim[g.i + 1] += g.d1;
    lim[g.i + 2] += g.d2;
}

// The same on limbs shared by a workgroup (LDS), by integer atomics.
__device__ __forceinline__ void exact_add_atomic(unsigned long long *lim, double x)
{
    const ExactDigits g = exact_digits(x, false);
    atomicAdd(lim + g.i, (unsigned long long)g.d0);
    atomicAdd(lim + g.i + 1, (unsigned long long)g.d1);
    atomicAdd(lim + g.i + 2, (unsigned long long)g.d2);
}

// Carry every limb into [0, 2^32); returns the final carry (0, or -1 for a
// negative sum in two's complement).
__device__ __forceinline__ int64_t exact_normalize(int64_t *lim)
{
    int64_t carry = 0;
    for (int k = 0; k < XL; ++k) {
        const int64_t v = lim[k] + carry;
        lim[k] = v & 0xffffffffll;
        carry = v >> 32;  // arithmetic shift: floor division by 2^32
    }
    return carry;
}

// The sum held by normalized limbs and their final carry, rounded once to
// binary64 (nearest, ties to even; an exact zero is +0).  Destroys lim.
__device__ __forceinline__ double exact_round_normalized(int64_t *lim, int64_t carry)
{
    const bool neg = carry < 0;
    if (neg) {  // magnitude = 2^(32 XL) - digits
        int64_t c = 1;
        for (int k = 0; k < XL; ++k) {
            const int64_t v = (~lim[k] & 0xffffffffll) + c;
            lim[k] = v & 0xffffffffll;
            c = v >> 32;
        }
    }
    int top = XL - 1;
    while (top >= 0 && lim[top] == 0) --top;
    if (top < 0) return 0.0;
    const int b = 32 * top + (32 - __builtin_clz((uint32_t)lim[top]));  // bit length of the magnitude
    double r;
    if (b <= 53) {  // exact: subnormal, or normal with at most 53 bits
        const uint64_t v = (uint64_t)lim[0] | (top >= 1 ? (uint64_t)lim[1] << 32 : 0ull);
        r = ldexp((double)v, -1074);
    } else {
        // T: the 64 bits below the leading one (inclusive); sticky: any lower bit
        const int s = b - 64;
        uint64_t T;
        bool sticky = false;
        if (s <= 0) {
            T = ((uint64_t)lim[0] | ((uint64_t)lim[1] << 32)) << (-s);
        } else {
            const int w = s >> 5, q = s & 31;
            const uint64_t x = (uint64_t)lim[w] | ((uint64_t)lim[w + 1] << 32);
            const uint64_t y = w + 2 < XL ? (uint64_t)lim[w + 2] : 0ull;
            T = q ? (x >> q) | (y << (64 - q)) : x;
            sticky = q && ((uint64_t)lim[w] & ((1ull << q) - 1)) != 0;
            for (int k = 0; k < w; ++k) sticky |= lim[k] != 0;
        }
        uint64_t mant = T >> 11;
        const uint64_t rest = T & 0x7ff;
        if ((rest & 0x400) && ((rest & 0x3ff) || sticky || (mant & 1))) ++mant;
        int e = b - 53;
        if (mant == (1ull << 53)) {
            mant >>= 1;
            ++e;
        }
        r = ldexp((double)mant, e - 1074);  // exact, or overflow to infinity
    }
    return neg ? -r : r;
}

__device__ __forceinline__ double exact_round(int64_t *lim)
{
    const int64_t c = exact_normalize(lim);
    return exact_round_normalized(lim, c);
}

// Result of a sum with non-finite terms (counts n_nan, n_pinf, n_ninf), or
// false when every term is finite.
__device__ __forceinline__ bool exact_special(int n_nan, int n_pinf, int n_ninf, double *out)
{
    if (n_nan || (n_pinf && n_ninf)) {
        *out = __longlong_as_double(0x7ff8000000000000ll);
        return true;
    }
    if (n_pinf) {
        *out = __longlong_as_double(0x7ff0000000000000ll);
        return true;
    }
    if (n_ninf) {
        *out = __longlong_as_double((long long)0xfff0000000000000ull);
        return true;
    }
    return false;
}

// Special-value class of x: 0 NaN, 1 +inf, 2 -inf, -1 finite.
__device__ __forceinline__ int exact_class(double x)
{
    if (x != x) return 0;
    if (x == __longlong_as_double(0x7ff0000000000000ll)) return 1;
    if (x == __longlong_as_double((long long)0xfff0000000000000ull)) return 2;
    return -1;
}

}  // namespace ea
