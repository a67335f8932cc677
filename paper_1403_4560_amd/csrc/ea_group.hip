// ea_group.hip -- per-class kernels of the walker-interleaved LDS engine
// (ea_group.hpp).
#include "ea_group.hpp"

namespace ea {

// VAR only separates the symbol of the one-sample-per-launch comparator.
template <int L, int JK, int VAR>
__global__ void __launch_bounds__(GROUP_MAX_THREADS, 4) group_sweep_kernel(SweepArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (int item = blockIdx.x; item < A.n_items; item += gridDim.x) {
        const int code = A.items[item];
        run_group_item<L, JK>(A, sample_of_item(A.samples, code >> 1), code & 1, smem);
    }
}

#define EA_GROUP(Lv)                                                 \
    template __global__ void group_sweep_kernel<Lv, 0, 0>(SweepArgs); \
    template __global__ void group_sweep_kernel<Lv, 1, 0>(SweepArgs); \
    template __global__ void group_sweep_kernel<Lv, 0, 1>(SweepArgs); \
    template __global__ void group_sweep_kernel<Lv, 1, 1>(SweepArgs);
EA_GROUP(2)
EA_GROUP(4)
EA_GROUP(6)
EA_GROUP(8)
EA_GROUP(10)
EA_GROUP(12)
EA_GROUP(14)
EA_GROUP(16)
#undef EA_GROUP

}  // namespace ea
