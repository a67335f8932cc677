// ea_finalize.hip -- disorder averages and jackknife errors of the observables
// of eqs. 3-6 on the device, from the per-slot accumulators of the selected
// samples of one system, with exact sums over samples (ea_exact.hpp).
#include "ea_exact.hpp"
#include "ea_types.hpp"

namespace ea {

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
