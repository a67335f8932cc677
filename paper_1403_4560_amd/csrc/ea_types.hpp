// ea_types.hpp -- layouts shared by the host library and the gfx950 kernels.
//
// Device memory of an ensemble (all offsets precomputed on the host):
//   spins   int8   per sample [2 chains][n_T walkers][2 parities][N/2]
//                  (walker order; a walker's bytes never move, exchanges
//                  permute the walker <-> slot maps instead)
//   Jsub    float  per sample [2 parities][3 directions][N/2] (Gaussian), or
//           int8   the same shape for +-1 couplings.  Jsub[p][d][h] is the
//                  bond from the parity-p site with sublattice index h to its
//                  +d neighbour.
//   per (sample, chain, slot or walker), index 2*slot_off + r*n_T + t:
//           walker_at_slot int32, EJ int64 (coupling energy in units of
//           2^-18 for Gaussian couplings, 1 for +-1), M int32 (magnetisation,
//           per walker), flips int64 and swaps int64 (per slot / pair)
//   per (sample, slot), index slot_off + t: beta float64, beta32 float32,
//           acc float64[36], lut uint32[2][7] (+-1 couplings)
//   frames  uint32 snapshot frames of both chains in slot order, one frame per
//                  measurement in a chunk, one bit per spin: frame f, sample s
//                  at word f*frame_words + frame_off[s], layout [2][n_T][L*L]
//                  rows, row (y, z) at index y + L z, bit x set iff s = -1
//   frameE  float64 [frame][2*total_slots] energies of the snapshotted walkers
//   Jbits   uint32 (+-1 couplings on the bit engine) per sample [2 parities]
//                  [6 bonds: +x, -x, +y, -y, +z, -z][N/64]: bit j of word g is
//                  set iff the bond of the parity-p site with sublattice index
//                  32 g + j in that direction is -1
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ea {

constexpr int NACC = 36;
constexpr int NPLANE = 9;
constexpr int MAX_T = 64;     // temperature slots per sample
constexpr int MAX_L = 32;     // a row of spins fits one 32-bit snapshot word
constexpr int LDS_MAX_L = 16; // largest lattice of the LDS-resident tier
constexpr int ROW_MAX_THREADS = 768;  // row engine: one thread per (walker, column)
constexpr int GROUP_MAX_THREADS = 512;  // group engine workgroup size cap

struct SampleDev {
    int32_t L;
    int32_t n_T;
    uint32_t sample_id;
    float h32;
    int64_t spin_off;   // bytes into spins (and into each frame)
    int64_t J_off;      // elements into Jsub
    int32_t slot_off;   // sum of n_T over earlier samples
    int32_t tier;       // 0 = LDS-resident, 1 = HBM-resident
    int64_t frame_off;  // words into each snapshot frame
    uint32_t down_mask; // +-1 couplings: bit a*7+b set iff 2 s (S_J + h) <= 0, s = 2a-1, S_J = 2b-6
    int32_t hgrid;      // Gaussian couplings: the field on the 2^-18 grid, round(h 2^18) within +-6 2^21
    int64_t jb_off;     // bit engine: words into Jbits
};

struct SweepArgs {
    const SampleDev *samples;
    const int32_t *items;       // (sample << 1) | chain, one per workgroup
    int32_t n_items;
    int32_t K;                  // sweeps in this launch
    int8_t *spins;
    const void *J;
    const double *beta;
    const float *beta32;
    const uint32_t *lut;
    int32_t *was;
    int64_t *EJ;
    int32_t *M;
    int64_t *flips;
    int64_t *swaps;
    uint32_t *frames;
    double *frameE;
    int64_t frame_words;
    int64_t total_slots;
    const int64_t *state;       // [0] sweeps completed before this launch
    uint32_t key0, key1;
    int32_t measure_every;
    int32_t pad;
    int64_t measure_start;
    // HBM-resident tier (one launch per half-sweep / exchange / snapshot)
    const int32_t *walkers;     // (sample << 7) | (chain << 6) | walker-or-slot
    int32_t n_walkers;
    int32_t p;                  // parity of this half-sweep
    int32_t it;                 // sweep index within the chunk: n = state[0] + it
    int32_t jkind;              // 0 Gaussian (energy unit 2^-18), 1 +-1 (unit 1)
    int64_t *dEJ;               // per walker: coupling-energy change of this sweep
    int32_t *dM;                // per walker: magnetisation change of this sweep
    int32_t *sow;               // per walker: its slot during this sweep
    const int32_t *Ju;          // Gaussian couplings as int32 multiples of 2^-18, Jsub layout
    const uint32_t *Jbits;      // bit engine: per sample [2 parities][6 bonds][N/64] words
};

struct MeasureArgs {
    const SampleDev *samples;
    const int32_t *slots;        // global slot indices of this launch (one lattice size)
    const int32_t *slot_sample;  // global slot -> sample
    const uint32_t *frames;
    const double *frameE;
    int64_t frame_words;
    int64_t total_slots;
    double *acc;
    const double *costab;        // [MAX_L + 1][MAX_L]: cos(2 pi c / L)
    const double *sintab;
    const int64_t *state;
    int32_t K;                   // chunk length (frames derived from state)
    int32_t explicit_frames;     // > 0: measure this many frames regardless
    int32_t measure_every;
    int32_t pad;
    int64_t measure_start;
};

// Batch launch (ea_batch.hip): one launch runs the work items of every
// lattice-size class of the small LDS-resident engines.  A unit is up to P
// items of one class that P equal, wave-aligned teams of a workgroup run side
// by side; one workgroup per unit, units ordered by decreasing cost (longest
// first), so no class waits for another's tail.
enum { BATCH_SITE = 0, BATCH_ROW = 1, BATCH_GROUP = 2 };
constexpr int BATCH_THREADS = 512;

struct BatchUnit {
    int32_t kind;   // engine << 8 | L
    int32_t first;  // index of the unit's first item in the item list
    int32_t count;  // real items, 1 .. P; teams beyond count run ghosts
    int32_t P;      // teams (threads per team: BATCH_THREADS / P)
    int32_t lds;    // LDS bytes per team (a multiple of 16)
    int32_t pad[3];
};

struct BatchArgs {
    const BatchUnit *units;
    int32_t n_units;
    int32_t pad;
    int32_t *counter;  // reserved
};

// Number of measurement sweeps among completed-sweep counts 1..x.
__host__ __device__ inline int64_t measurements_upto(int64_t x, int32_t m, int64_t start)
{
    if (m <= 0 || x <= start) return 0;
    return (x - start) / m;
}

// The first completed-sweep count beyond x at which a measurement is taken:
// the least start + k m > x with k >= 1 (INT64_MAX if m <= 0).  Sweep loops
// step it by m instead of testing every count with a 64-bit division.
__host__ __device__ inline int64_t next_measurement(int64_t x, int32_t m, int64_t start)
{
    if (m <= 0) return INT64_MAX;
    return start + (measurements_upto(x, m, start) + 1) * m;
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS layout of one LDS-tier work item (bytes).  Shared with the host, which
// sizes the dynamic LDS of a launch with lds_total().
struct LdsOff {
    size_t spins, J, was, sow, M, dM, fl, sw, EJ, dEJ, lut, b32, b64, total;
};

// Bytes between consecutive walkers of the per-item frame's LDS spins: N plus
// 8.  The row engine's wave holds the same columns of four walkers, whose words
// fall two words (mod 4) apart, so the two walkers of each half-wave read
// disjoint LDS banks.
__host__ __device__ inline size_t item_walker_stride(int L) { return (size_t)L * L * L + 8; }

__host__ __device__ inline LdsOff lds_offsets(int L, int nT, int jkind)
{
    const size_t N = (size_t)L * L * L;
    const size_t T4 = (size_t)((nT + 3) & ~3);
    LdsOff o;
    o.spins = 0;
    o.J = align16((size_t)nT * item_walker_stride(L));
    o.was = o.J + align16(3 * N * (jkind == 0 ? 4 : 1));
    o.sow = o.was + 4 * T4;
    o.M = o.sow + 4 * T4;
    o.dM = o.M + 4 * T4;
    o.fl = o.dM + 4 * T4;
    o.sw = o.fl + 4 * T4;
    o.EJ = align16(o.sw + 4 * T4);
    o.dEJ = o.EJ + 8 * T4;
    o.lut = o.dEJ + 8 * T4;
    o.b32 = o.lut + (jkind == 1 ? 4 * 14 * T4 : 0);
    o.b64 = align16(o.b32 + 4 * T4);
    o.total = align16(o.b64 + 8 * T4);
    return o;
}

// LDS layout of one bit-engine work item (bytes): the 256-entry
// bit-to-byte spreading table and the per-slot threshold tables [n_T][8] at
// fixed offsets, then spin bits [n_T][2][N/64] words, bond bits [2][6][N/64],
// then the per-walker/slot arrays of the common frame.
struct BitsLdsOff {
    size_t spread, th, spins, J, was, sow, M, dM, fl, sw, EJ, dEJ, b64, total;
};

__host__ __device__ inline BitsLdsOff bits_lds_offsets(int L, int nT)
{
    const size_t G = (size_t)L * L * L / 64;
    const size_t T4 = (size_t)((nT + 3) & ~3);
    BitsLdsOff o;
    o.spread = 0;
    o.th = 256 * 8;
    o.spins = align16(o.th + (size_t)nT * 8 * 4);
    o.J = o.spins + (size_t)nT * 2 * G * 4;
    o.was = o.J + 12 * G * 4;
    o.sow = o.was + 4 * T4;
    o.M = o.sow + 4 * T4;
    o.dM = o.M + 4 * T4;
    o.fl = o.dM + 4 * T4;
    o.sw = o.fl + 4 * T4;
    o.EJ = align16(o.sw + 4 * T4);
    o.dEJ = o.EJ + 8 * T4;
    o.b64 = o.dEJ + 8 * T4;
    o.total = align16(o.b64 + 8 * T4);
    return o;
}

// LDS layout of one group-engine work item (bytes): quad words
// [2][ceil(n_T/4)][N/2 + 1], couplings (int32 units of 2^-18, or int8 +-1)
// [2][3][N/2], the neighbour table [N/2] (16 B per site), +-1 threshold
// tables [n_T][14], then the per-walker/slot arrays of the common frame.
struct GroupLdsOff {
    size_t spins, J, nb, lut, was, sow, M, dM, fl, sw, EJ, dEJ, b32, b64, total;
};

__host__ __device__ inline GroupLdsOff group_lds_offsets(int L, int nT, int jkind)
{
    const size_t N = (size_t)L * L * L, NQ = (size_t)(nT + 3) / 4;
    const size_t T4 = (size_t)((nT + 3) & ~3);
    GroupLdsOff o;
    o.spins = 0;
    o.J = align16(2 * NQ * (N / 2 + 1) * 4);
    o.nb = align16(o.J + 3 * N * (jkind == 0 ? 4 : 1));
    o.lut = o.nb + (N / 2) * 16;
    o.was = o.lut + (jkind == 1 ? 4 * 14 * T4 : 0);
    o.sow = o.was + 4 * T4;
    o.M = o.sow + 4 * T4;
    o.dM = o.M + 4 * T4;
    o.fl = o.dM + 4 * T4;
    o.sw = o.fl + 4 * T4;
    o.EJ = align16(o.sw + 4 * T4);
    o.dEJ = o.EJ + 8 * T4;
    o.b32 = o.dEJ + 8 * T4;
    o.b64 = align16(o.b32 + 4 * T4);
    o.total = align16(o.b64 + 8 * T4);
    return o;
}

// Threads per walker of the bit engine: the largest power of two <= 64 that
// divides the N/64 words of a sublattice and keeps n_T * TPW <= 1024.
__host__ __device__ inline int bits_tpw(int L, int nT)
{
    const int G = L * L * L / 64;
    int t = 64;
    while (t > 1 && (t > G || nT * t > 1024)) t >>= 1;
    return t;
}

}  // namespace ea
