// ea_batch.hip -- one launch for the lattice-size classes of the
// small LDS-resident engines (group engine at any even L <= 16, row engine at
// L = 8, site engine at L = 2 and 4, the chains too small for the group
// engine), so that a batch of uneven sizes (Table I runs several
// L; its samples are independent) runs as one launch per chunk of sweeps
// instead of one launch per size with a tail each.
//
// Every workgroup has BATCH_THREADS threads and runs one unit: the unit's P
// teams each run one work item of the unit's class (the same code as the
// class's own kernel, on the team's threads and LDS region), and every team
// passes the same barriers because every item of a chunk runs the same sweeps
// and measurements.  A unit with fewer items than teams fills the rest with
// ghost teams (a copy of its first item that writes nothing back).  Units are
// ordered longest first; which workgroup runs a unit does not change any
// result.  (A persistent form, workgroups looping over a queue of units, let
// the compiler hoist every engine's loop invariants out of the queue loop,
// where they stayed live together and spilled; measured slower.)
#include "ea_group.hpp"
#include "ea_row.hpp"

namespace ea {

template <int JK>
__device__ __forceinline__ void batch_dispatch(const SweepArgs &A, int kind, const SampleDev &d, int r, char *mem,
                                               const Team tm)
{
#define EA_G(Lv) \
    case (BATCH_GROUP << 8) | Lv: run_group_item<Lv, JK>(A, d, r, mem, tm); break;
#define EA_S(Lv) \
    case (BATCH_SITE << 8) | Lv: run_item<Lv, JK, false>(A, d, r, mem, tm); break;
    switch (kind) {
        EA_G(2) EA_G(4) EA_G(6) EA_G(8) EA_G(10) EA_G(12) EA_G(14) EA_G(16)
        EA_S(2) EA_S(4)
    case (BATCH_ROW << 8) | 8:
        if constexpr (JK == 0) run_item<8, 0, true>(A, d, r, mem, tm);
        break;
    default: break;
    }
#undef EA_G
#undef EA_S
}

// Held to 128 VGPRs (four waves per SIMD), as the class kernels of these
// engines are.  One workgroup per unit: the units are ordered longest first,
// and the hardware dispatcher hands workgroups to compute units in that order
// as resident ones finish, which deals the units out as list scheduling with
// longest-first priority would.
template <int JK>
__global__ void __launch_bounds__(BATCH_THREADS, 4) batch_sweep_kernel(SweepArgs A, BatchArgs B)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int u = blockIdx.x;
    if (u >= B.n_units) return;
    const BatchUnit U = B.units[u];
    const int T = BATCH_THREADS / U.P;
    const int team = __builtin_amdgcn_readfirstlane((int)threadIdx.x / T);
    const Team tm{(int)threadIdx.x - team * T, T, team >= U.count};
    const int code = A.items[U.first + (team < U.count ? team : 0)];
    batch_dispatch<JK>(A, U.kind, sample_of_item(A.samples, code >> 1), code & 1, smem + (size_t)team * U.lds, tm);
}

template __global__ void batch_sweep_kernel<0>(SweepArgs, BatchArgs);
template __global__ void batch_sweep_kernel<1>(SweepArgs, BatchArgs);

}  // namespace ea
