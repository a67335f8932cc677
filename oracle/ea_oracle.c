/*
 * ea_oracle.c -- plain, slow CPU oracle for Metropolis Monte Carlo with
 * parallel tempering on the three-dimensional Edwards-Anderson spin glass in a
 * uniform external field.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library; the two meet only through the seeded input arrays.
 *
 * What is computed, and where it comes from (arXiv:1403.4560):
 *   - Hamiltonian H = -sum_<ij> J_ij S_i S_j - h sum_i S_i on a periodic simple
 *     cubic lattice of N = L^3 sites               (Methods, eq. 1)
 *   - bimodal or Gaussian couplings                (Methods; Conclusion)
 *   - single-spin-flip Monte Carlo with parallel tempering over N_T
 *     temperatures, two independent replicas per temperature
 *                                                  (Methods, paragraph on PT)
 *   - overlap q(k) = (1/N) sum_j S_j^a S_j^b e^{i k.r_j}   (Methods, eq. 2)
 *     measured at k = 0, at the three axis vectors of length 2pi/L and at the
 *     six images of (2pi/L, 2pi/L, 0)              (eqs. 4-6; point-group
 *                                                   averaging in Results)
 * Where the paper is silent the numeric contract below fixes one reading
 * (Metropolis rule, checkerboard order, Philox4x32-10 counter map, in-house
 * exponentials, swap schedule); each reading is listed in the design notes.
 *
 * Numeric contract ("mirror" mode, bit-exact against the GPU path):
 *   site i = x + L(y + Lz), parity p = (x+y+z)&1, sublattice index h = i>>1.
 *   bond J_d[i] couples i and i + d (periodic); d = 0,1,2 for x,y,z.
 *   field  S_J = sum of J*s over +x,-x,+y,-y,+z,-z   (exact: J on a 2^-18 grid)
 *   f = fl32(S_J + h32), dE = 2 s_i f, x = -fl32(beta32[t] * dE)
 *   Philox4x32-10, key = (seed lo, seed hi),
 *     counter = (h>>2, 2n+p, (0<<28)|(t<<1)|r, sample_id), word h&3
 *   u24 = (word>>8) * 2^-24;  accept iff dE <= 0 or u24 < exp_ea32(x)
 *   +-J couplings: accept iff dE64 <= 0 or word < thr[t][s_i][S_J], with
 *     thr = min(2^32-1, floor(2^32 exp(-beta[t] dE64))), dE64 = 2 s (S_J + h32)
 *   after both half-sweeps of sweep n, per chain r: even-odd replica exchange
 *     on pairs (t, t+1), t = n&1, n&1 + 2, ...:
 *     D = fl64(fl64(beta[t]-beta[t+1]) * fl64(E(w_t) - E(w_t+1)))
 *     accept iff D >= 0 or u53 < exp_ea64(D);
 *     u53 from Philox counter (0, n, (1<<28)|(t<<1)|r, sample_id), words 0,1
 *   measurement after sweep n iff m > 0, n+1 > start, (n+1-start) % m == 0.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared (no FMA, SSE
 * arithmetic, round-to-nearest-even).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EAO_NACC 36   /* accumulators per (sample, slot); layout in eao_measure */
#define EAO_NPLANE 9  /* plane-sum families: 3 axes + 6 diagonals */

enum { EAO_J_GAUSS = 0, EAO_J_PM1 = 1 };
enum { EAO_MODE_MIRROR = 0, EAO_MODE_FP64 = 1 };

static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static double u2d(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror & Shaw, "Parallel Random Numbers: As
 * Easy as 1, 2, 3", SC'11.  One round multiplies counter words 0 and 2 by the
 * two round multipliers into 64-bit products and mixes the high halves with
 * the other two counter words and the key; the key is advanced by the two Weyl
 * increments between rounds. */
void eao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* exp_ea32: e^x for x <= 0 in binary32 by Cody & Waite argument reduction
 * (Software Manual for the Elementary Functions, 1980) and a degree-7 Taylor
 * polynomial in Horner form.  Every operation is one IEEE binary32 operation,
 * rounded to nearest even; nothing is fused.
 *   x < -86          -> 0
 *   k = rint(x * LOG2E)                   LOG2E = fl32(1/ln 2)
 *   r = (x - k*C1) - k*C2                 C1 = fl32(ln 2) with 8 low bits
 *                                         cleared, C2 = fl32(ln 2 - C1)
 *   P = 1/7!, then P = P*r + 1/j! for j = 6..0   (coefficients fl32(1/j!))
 *   result = P * 2^k  (exact: the result is a normal number)            */
float eao_exp_ea32(float x)
{
    const float LOG2E = u2f(0x3FB8AA3Bu);
    const float C1 = u2f(0x3F317200u);
    const float C2 = u2f(0x35BFBE8Eu);
    const float P[8] = { u2f(0x3F800000u), u2f(0x3F800000u), u2f(0x3F000000u),
                         u2f(0x3E2AAAABu), u2f(0x3D2AAAABu), u2f(0x3C088889u),
                         u2f(0x3AB60B61u), u2f(0x39500D01u) };
    if (x < -86.0f)
        return 0.0f;
    float t = x * LOG2E;
    float k = rintf(t);
    float kc1 = k * C1;
    float r = x - kc1;
    float kc2 = k * C2;
    r = r - kc2;
    float p = P[7];
    for (int j = 6; j >= 0; --j) {
        float pr = p * r;
        p = pr + P[j];
    }
    return ldexpf(p, (int)k);
}

/* exp_ea64: the same construction in binary64.  x < -700 -> 0; C1 = fl64(ln 2)
 * with 11 low bits cleared, C2 = fl64(ln 2 - C1), degree-13 Taylor polynomial
 * with coefficients fl64(1/j!). */
double eao_exp_ea64(double x)
{
    const double LOG2E = u2d(0x3FF71547652B82FEull);
    const double C1 = u2d(0x3FE62E42FEFA3800ull);
    const double C2 = u2d(0x3D2EF35793C76730ull);
    const double Q[14] = {
        u2d(0x3FF0000000000000ull), u2d(0x3FF0000000000000ull), u2d(0x3FE0000000000000ull),
        u2d(0x3FC5555555555555ull), u2d(0x3FA5555555555555ull), u2d(0x3F81111111111111ull),
        u2d(0x3F56C16C16C16C17ull), u2d(0x3F2A01A01A01A01Aull), u2d(0x3EFA01A01A01A01Aull),
        u2d(0x3EC71DE3A556C734ull), u2d(0x3E927E4FB7789F5Cull), u2d(0x3E5AE64567F544E4ull),
        u2d(0x3E21EED8EFF8D898ull), u2d(0x3DE6124613A86D09ull) };
    if (x < -700.0)
        return 0.0;
    double t = x * LOG2E;
    double k = rint(t);
    double kc1 = k * C1;
    double r = x - kc1;
    double kc2 = k * C2;
    r = r - kc2;
    double p = Q[13];
    for (int j = 12; j >= 0; --j) {
        double pr = p * r;
        p = pr + Q[j];
    }
    return ldexp(p, (int)k);
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry (Methods: simple cubic, periodic boundaries). */
static int wrap(int a, int L) { return ((a % L) + L) % L; }
static int site_at(int L, int x, int y, int z)
{
    return wrap(x, L) + L * (wrap(y, L) + L * wrap(z, L));
}

/* Coupling value of bond d at site i (bond between i and i + d). */
static double bond(int jkind, const void *J, int N, int d, int i)
{
    if (jkind == EAO_J_GAUSS)
        return (double)((const float *)J)[d * N + i];
    return (double)((const int8_t *)J)[d * N + i];
}

/* The six neighbours of site i in the order +x,-x,+y,-y,+z,-z, with the bond
 * that joins each one to i.  Bond +d is J_d[i]; bond -d is J_d[i - d]. */
static void neighbours(int L, int i, int nb[6], int bsite[6], int bdir[6])
{
    int x = i % L, y = (i / L) % L, z = i / (L * L);
    nb[0] = site_at(L, x + 1, y, z); bsite[0] = i;     bdir[0] = 0;
    nb[1] = site_at(L, x - 1, y, z); bsite[1] = nb[1]; bdir[1] = 0;
    nb[2] = site_at(L, x, y + 1, z); bsite[2] = i;     bdir[2] = 1;
    nb[3] = site_at(L, x, y - 1, z); bsite[3] = nb[3]; bdir[3] = 1;
    nb[4] = site_at(L, x, y, z + 1); bsite[4] = i;     bdir[4] = 2;
    nb[5] = site_at(L, x, y, z - 1); bsite[5] = nb[5]; bdir[5] = 2;
}

/* Exact coupling energy E_J = -sum over the 3N bonds of J_d[i] s_i s_{i+d}
 * and magnetisation M = sum_i s_i of one configuration (eq. 1).  On the 2^-18
 * grid every partial sum is exact in binary64. */
void eao_energy(int32_t L, int32_t jkind, const void *J, const int8_t *s,
                double *EJ, int32_t *M)
{
    int N = L * L * L;
    double e = 0.0;
    int32_t m = 0;
    for (int i = 0; i < N; ++i) {
        int x = i % L, y = (i / L) % L, z = i / (L * L);
        int nx = site_at(L, x + 1, y, z), ny = site_at(L, x, y + 1, z),
            nz = site_at(L, x, y, z + 1);
        e -= bond(jkind, J, N, 0, i) * s[i] * s[nx];
        e -= bond(jkind, J, N, 1, i) * s[i] * s[ny];
        e -= bond(jkind, J, N, 2, i) * s[i] * s[nz];
        m += s[i];
    }
    *EJ = e;
    *M = m;
}

/* Local field S_J(i) = sum_j J_ij s_j over the six neighbours in the fixed
 * order +x,-x,+y,-y,+z,-z, in binary32 (exact on the 2^-18 grid). */
static float field32(int L, int jkind, const void *J, const int8_t *s, int i)
{
    int N = L * L * L, nb[6], bs[6], bd[6];
    neighbours(L, i, nb, bs, bd);
    float S = 0.0f;
    for (int k = 0; k < 6; ++k) {
        float Jk = (float)bond(jkind, J, N, bd[k], bs[k]);
        float term = Jk * (float)s[nb[k]];
        S = S + term;
    }
    return S;
}

/* Metropolis threshold table for +-1 couplings: thr[t][a][b], a = (s_i+1)/2,
 * b = (S_J+6)/2, S_J in {-6,...,6}.  Host binary64 with libm exp. */
static void pm1_thresholds(int n_T, const double *beta, float h32, uint32_t *thr)
{
    for (int t = 0; t < n_T; ++t)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 7; ++b) {
                double si = a ? 1.0 : -1.0;
                double SJ = (double)(2 * b - 6);
                double dE = 2.0 * si * (SJ + (double)h32);
                uint32_t v;
                if (dE <= 0.0) {
                    v = 0xFFFFFFFFu;
                } else {
                    double p = ldexp(exp(-beta[t] * dE), 32);
                    v = p >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)floor(p);
                }
                thr[(t * 2 + a) * 7 + b] = v;
            }
}

/* ------------------------------------------------------------------------ */
/* Measurement of one slot (eq. 2 at k = 0, the axis vectors and the six
 * images of (2pi/L,2pi/L,0)); accumulator layout per slot:
 *   [0] n            [1..4] sum q0, q0^2, q0^3, q0^4
 *   [5+3f .. 7+3f]   for plane family f = 0..8: sum Re q(k_f), sum Im q(k_f),
 *                    sum |q(k_f)|^2.  f = 0,1,2: k along x,y,z;
 *                    f = 3..8: k = (1,1,0),(1,-1,0),(1,0,1),(1,0,-1),
 *                    (0,1,1),(0,1,-1) times 2pi/L
 *   [32,33]          sum E, E^2 of the chain-a walker at this slot
 *   [34,35]          sum E, E^2 of the chain-b walker
 * The plane coordinate of site (x,y,z) for family f is c = k_f.r mod L.
 * Re = (sum_c P[c] cos(2pi c/L)) / N summed in c order (Im with sin).     */
static int plane_coord(int f, int L, int x, int y, int z)
{
    switch (f) {
    case 0: return x;
    case 1: return y;
    case 2: return z;
    case 3: return wrap(x + y, L);
    case 4: return wrap(x - y, L);
    case 5: return wrap(x + z, L);
    case 6: return wrap(x - z, L);
    case 7: return wrap(y + z, L);
    default: return wrap(y - z, L);
    }
}

/* Integer sums of one overlap field: S0 = sum q_i and P_f[c] (f-major). */
static void overlap_sums(int L, const int8_t *sa, const int8_t *sb, int32_t *S0,
                         int32_t *P /* [9][L] */)
{
    int N = L * L * L;
    memset(P, 0, sizeof(int32_t) * EAO_NPLANE * L);
    int32_t s0 = 0;
    for (int i = 0; i < N; ++i) {
        int q = sa[i] * sb[i];
        int x = i % L, y = (i / L) % L, z = i / (L * L);
        s0 += q;
        for (int f = 0; f < EAO_NPLANE; ++f)
            P[f * L + plane_coord(f, L, x, y, z)] += q;
    }
    *S0 = s0;
}

static void accumulate(int L, int32_t S0, const int32_t *P, double Ea, double Eb,
                       const double *cosc, const double *sinc, double *acc)
{
    double N = (double)(L * L * L);
    double q0 = (double)S0 / N;
    acc[0] += 1.0;
    acc[1] += q0;
    acc[2] += q0 * q0;
    acc[3] += (q0 * q0) * q0;
    acc[4] += (q0 * q0) * (q0 * q0);
    for (int f = 0; f < EAO_NPLANE; ++f) {
        double re = 0.0, im = 0.0;
        for (int c = 0; c < L; ++c) {
            re += (double)P[f * L + c] * cosc[c];
            im += (double)P[f * L + c] * sinc[c];
        }
        re = re / N;
        im = im / N;
        acc[5 + 3 * f] += re;
        acc[6 + 3 * f] += im;
        acc[7 + 3 * f] += re * re + im * im;
    }
    acc[32] += Ea;
    acc[33] += Ea * Ea;
    acc[34] += Eb;
    acc[35] += Eb * Eb;
}

/* Measurement of a single configuration pair; exported for hand-made cases. */
void eao_measure_pair(int32_t L, const int8_t *sa, const int8_t *sb, double Ea,
                      double Eb, double *acc /* [36] */, int32_t *sums /* [1+9L] */)
{
    double cosc[64], sinc[64];
    for (int c = 0; c < L; ++c) {
        double th = (2.0 * M_PI * (double)c) / (double)L;
        cosc[c] = cos(th);
        sinc[c] = sin(th);
    }
    int32_t S0, P[EAO_NPLANE * 64];
    overlap_sums(L, sa, sb, &S0, P);
    accumulate(L, S0, P, Ea, Eb, cosc, sinc, acc);
    if (sums) {
        sums[0] = S0;
        memcpy(sums + 1, P, sizeof(int32_t) * EAO_NPLANE * L);
    }
}

/* ------------------------------------------------------------------------ */
/* Run n_sweeps sweeps of one disorder sample (both chains, all slots).
 *
 * spins          [2][n_T][N] int8 +-1, indexed by walker (walkers never move)
 * walker_at_slot [2][n_T]    walker that currently sits at temperature slot t
 * EJ, M          [2][n_T]    per walker: coupling energy and magnetisation
 * sweep          sweeps completed so far (the Philox sweep counter)
 * acc            [n_T][36]   binary64 accumulators (see accumulate)
 * flips          [2][n_T]    accepted spin flips, counted at the slot held
 * swaps          [2][n_T]    accepted exchanges of pair (t, t+1), at index t
 * trace          optional [trace_cap][n_T][1+9L] integer sums per measurement
 * Returns 0, or -1 on invalid arguments.                                     */
int eao_run(int32_t L, int32_t n_T, const double *beta, float h32, int32_t jkind,
            const void *J, uint64_t seed, uint32_t sample_id, int32_t measure_every,
            int64_t measure_start, int32_t mode, int64_t n_sweeps,
            int8_t *spins, int32_t *walker_at_slot, double *EJ, int32_t *M,
            int64_t *sweep, double *acc, int64_t *flips, int64_t *swaps,
            int32_t *trace, int64_t trace_cap, int64_t *trace_len)
{
    if (L < 2 || L > 64 || (L & 1) || n_T < 1 || n_sweeps < 0)
        return -1;
    const int N = L * L * L;
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    float *beta32 = (float *)malloc(sizeof(float) * n_T);
    uint32_t *thr = (uint32_t *)malloc(sizeof(uint32_t) * n_T * 14);
    for (int t = 0; t < n_T; ++t)
        beta32[t] = (float)beta[t];
    if (jkind == EAO_J_PM1)
        pm1_thresholds(n_T, beta, h32, thr);
    double cosc[64], sinc[64];
    for (int c = 0; c < L; ++c) {
        double th = (2.0 * M_PI * (double)c) / (double)L;
        cosc[c] = cos(th);
        sinc[c] = sin(th);
    }
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * EAO_NPLANE * L);

    for (int64_t it = 0; it < n_sweeps; ++it) {
        const int64_t n = *sweep;
        /* Two half-sweeps: every site of parity 0, then every site of parity 1. */
        for (int p = 0; p < 2; ++p) {
            for (int r = 0; r < 2; ++r) {
                for (int t = 0; t < n_T; ++t) {
                    const int w = walker_at_slot[r * n_T + t];
                    int8_t *s = spins + ((size_t)r * n_T + w) * N;
                    for (int i = 0; i < N; ++i) {
                        int x = i % L, y = (i / L) % L, z = i / (L * L);
                        if (((x + y + z) & 1) != p)
                            continue;
                        const int hidx = i >> 1;
                        const int si = s[i];
                        const float SJ = field32(L, jkind, J, s, i);
                        int accept;
                        if (mode == EAO_MODE_MIRROR) {
                            uint32_t ctr[4] = { (uint32_t)(hidx >> 2), (uint32_t)(2 * n + p),
                                                (0u << 28) | ((uint32_t)t << 1) | (uint32_t)r,
                                                sample_id };
                            uint32_t word4[4];
                            eao_philox4x32_10(ctr, key, word4);
                            const uint32_t word = word4[hidx & 3];
                            if (jkind == EAO_J_PM1) {
                                double dE64 = 2.0 * (double)si * ((double)SJ + (double)h32);
                                int a = (si + 1) / 2, b = ((int)SJ + 6) / 2;
                                accept = dE64 <= 0.0 || word < thr[(t * 2 + a) * 7 + b];
                            } else {
                                float f = SJ + h32;
                                float dE = (2.0f * (float)si) * f;
                                if (dE <= 0.0f) {
                                    accept = 1;
                                } else {
                                    float xarg = -(beta32[t] * dE);
                                    float u24 = (float)(word >> 8) * 0x1p-24f;
                                    accept = u24 < eao_exp_ea32(xarg);
                                }
                            }
                        } else {
                            /* binary64 reference dynamics: field, energy change
                             * and acceptance in binary64 with libm exp and a
                             * 53-bit uniform from its own counter purpose (4). */
                            uint32_t ctr[4] = { (uint32_t)hidx, (uint32_t)(2 * n + p),
                                                (4u << 28) | ((uint32_t)t << 1) | (uint32_t)r,
                                                sample_id };
                            uint32_t word4[4];
                            eao_philox4x32_10(ctr, key, word4);
                            double u53 = ((double)(word4[0] >> 5) * 67108864.0 +
                                          (double)(word4[1] >> 6)) * 0x1p-53;
                            double dE = 2.0 * (double)si * ((double)SJ + (double)h32);
                            accept = dE <= 0.0 || u53 < exp(-beta[t] * dE);
                        }
                        if (accept) {
                            s[i] = (int8_t)(-si);
                            EJ[r * n_T + w] += 2.0 * (double)si * (double)SJ;
                            M[r * n_T + w] -= 2 * si;
                            flips[r * n_T + t] += 1;
                        }
                    }
                }
            }
        }
        /* Replica exchange between neighbouring temperatures, per chain. */
        for (int r = 0; r < 2; ++r) {
            for (int t = (int)(n & 1); t + 1 < n_T; t += 2) {
                int w0 = walker_at_slot[r * n_T + t], w1 = walker_at_slot[r * n_T + t + 1];
                double E0 = EJ[r * n_T + w0] - (double)h32 * (double)M[r * n_T + w0];
                double E1 = EJ[r * n_T + w1] - (double)h32 * (double)M[r * n_T + w1];
                double db = beta[t] - beta[t + 1];
                double dEn = E0 - E1;
                double D = db * dEn;
                int accept = D >= 0.0;
                if (!accept) {
                    uint32_t ctr[4] = { 0u, (uint32_t)n,
                                        (1u << 28) | ((uint32_t)t << 1) | (uint32_t)r, sample_id };
                    uint32_t word4[4];
                    eao_philox4x32_10(ctr, key, word4);
                    double u53 = ((double)(word4[0] >> 5) * 67108864.0 +
                                  (double)(word4[1] >> 6)) * 0x1p-53;
                    accept = u53 < eao_exp_ea64(D);
                }
                if (accept) {
                    walker_at_slot[r * n_T + t] = w1;
                    walker_at_slot[r * n_T + t + 1] = w0;
                    swaps[r * n_T + t] += 1;
                }
            }
        }
        *sweep = n + 1;
        /* Measurement of the two-replica overlap at every slot. */
        const int64_t done = n + 1;
        if (measure_every > 0 && done > measure_start &&
            (done - measure_start) % measure_every == 0) {
            for (int t = 0; t < n_T; ++t) {
                int wa = walker_at_slot[t], wb = walker_at_slot[n_T + t];
                const int8_t *sa = spins + (size_t)wa * N;
                const int8_t *sb = spins + ((size_t)n_T + wb) * N;
                double Ea = EJ[wa] - (double)h32 * (double)M[wa];
                double Eb = EJ[n_T + wb] - (double)h32 * (double)M[n_T + wb];
                int32_t S0;
                overlap_sums(L, sa, sb, &S0, P);
                accumulate(L, S0, P, Ea, Eb, cosc, sinc, acc + (size_t)t * EAO_NACC);
                if (trace && trace_len && *trace_len < trace_cap) {
                    int32_t *dst = trace + ((size_t)(*trace_len) * n_T + t) * (1 + EAO_NPLANE * L);
                    dst[0] = S0;
                    memcpy(dst + 1, P, sizeof(int32_t) * EAO_NPLANE * L);
                }
            }
            if (trace && trace_len && *trace_len < trace_cap)
                *trace_len += 1;
        }
    }
    free(P);
    free(thr);
    free(beta32);
    return 0;
}

/* Local energy change of flipping site i, in binary32 as the sweep computes it
 * (Gaussian couplings), exported for tests of the bookkeeping. */
float eao_delta_e32(int32_t L, int32_t jkind, const void *J, const int8_t *s,
                    float h32, int32_t i)
{
    float SJ = field32(L, jkind, J, s, i);
    float f = SJ + h32;
    return (2.0f * (float)s[i]) * f;
}

/* The +-J threshold table, exported for tests: [n_T][2][7]. */
void eao_pm1_thresholds(int32_t n_T, const double *beta, float h32, uint32_t *thr)
{
    pm1_thresholds(n_T, beta, h32, thr);
}

/* Array forms of the two exponentials, for exhaustive accuracy tests. */
void eao_exp_ea32_n(const float *x, float *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = eao_exp_ea32(x[i]);
}

void eao_exp_ea64_n(const double *x, double *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = eao_exp_ea64(x[i]);
}
