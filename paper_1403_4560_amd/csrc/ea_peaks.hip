// ea_peaks.hip -- microbenchmarks of the rates the sweep kernels' rooflines
// are priced against: the issue rate of the three VALU instruction kinds the
// Metropolis and Philox arithmetic is made of (a two-input xor stands for
// the simple ops, the 32x32->64 multiply-add and the 32-bit high multiply for
// the generator's products) and of the hardware exponential, LDS read
// bandwidth and HBM copy bandwidth.
//
// Each VALU kernel runs 16 independent dependency chains per lane, so issue,
// not latency, bounds it; the grid holds eight waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ea.h"

namespace ea {
namespace {

constexpr int PK_THREADS = 256;
constexpr int PK_CHAINS = 16;

// v_xor_b32: a_i <- a_i ^ b (one instruction per step, kept by the asm)
__global__ void __launch_bounds__(PK_THREADS) peak_xor_kernel(uint32_t *out, uint32_t seed, int rounds)
{
    uint32_t a[PK_CHAINS];
    const uint32_t b = seed ^ (threadIdx.x * 0x9E3779B9u);
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) a[i] = seed + i + blockIdx.x;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int i = 0; i < PK_CHAINS; ++i) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) x ^= a[i];
    out[blockIdx.x * PK_THREADS + threadIdx.x] = x;
}

// v_mad_u64_u32: a_i <- lo(a_i M + c), the Philox product with an add folded in
__global__ void __launch_bounds__(PK_THREADS) peak_mad64_kernel(uint32_t *out, uint32_t seed, int rounds)
{
    constexpr uint64_t M = 0xD2511F53u;
    uint32_t a[PK_CHAINS];
    const uint64_t c = seed ^ threadIdx.x;
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) a[i] = seed + i + blockIdx.x;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int i = 0; i < PK_CHAINS; ++i) a[i] = (uint32_t)((uint64_t)a[i] * M + c);
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) x ^= a[i];
    out[blockIdx.x * PK_THREADS + threadIdx.x] = x;
}

// v_mul_hi_u32: a_i <- hi(a_i M) + 1 is two ops; hi(a_i M_i) with the chain
// carried through the high half alone is one (M odd keeps it from collapsing
// within the run)
__global__ void __launch_bounds__(PK_THREADS) peak_mulhi_kernel(uint32_t *out, uint32_t seed, int rounds)
{
    uint32_t a[PK_CHAINS];
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) a[i] = 0x80000000u | (seed + 977u * i + blockIdx.x);
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int i = 0; i < PK_CHAINS; ++i)
            asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[i]) : "v"(0xFFFFFFF1u));
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) x ^= a[i];
    out[blockIdx.x * PK_THREADS + threadIdx.x] = x;
}

// v_exp_f32: a_i <- 2^(-a_i) stays in (0.5, 1) (the hardware exponential of
// the acceptance estimate)
__global__ void __launch_bounds__(PK_THREADS) peak_exp_kernel(uint32_t *out, uint32_t seed, int rounds)
{
    float a[PK_CHAINS];
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) a[i] = 0.5f + (float)((seed + i + threadIdx.x) & 255u) * 0x1p-9f;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int i = 0; i < PK_CHAINS; ++i) asm volatile("v_exp_f32 %0, -%0" : "+v"(a[i]));
    }
    float x = 0.f;
#pragma unroll
    for (int i = 0; i < PK_CHAINS; ++i) x += a[i];
    out[blockIdx.x * PK_THREADS + threadIdx.x] = __float_as_uint(x);
}

// LDS reads: 16 bytes per lane per read, consecutive lanes on consecutive
// 16-byte slots (no bank conflicts), eight reads per round at fixed offsets
// covering the 32 KB buffer; two three-input xors per read keep the data live
// (the memory clobber makes every round read again)
constexpr int PK_LDS_SLOTS = 8 * PK_THREADS;  // uint4 slots, 32 KB
__global__ void __launch_bounds__(PK_THREADS) peak_lds_kernel(uint32_t *out, uint32_t seed, int rounds)
{
    __shared__ uint4 buf[PK_LDS_SLOTS];
    for (int i = threadIdx.x; i < PK_LDS_SLOTS; i += PK_THREADS)
        buf[i] = make_uint4(seed + i, seed ^ i, seed * i, seed - i);
    __syncthreads();
    uint32_t x0 = 0, x1 = 0;
    const uint4 *p = buf + threadIdx.x;
    for (int r = 0; r < rounds; ++r) {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint4 v = p[u * PK_THREADS];
            x0 = __builtin_amdgcn_bitop3_b32(x0, v.x, v.y, 0x96);
            x1 = __builtin_amdgcn_bitop3_b32(x1, v.z, v.w, 0x96);
        }
    }
    out[blockIdx.x * PK_THREADS + threadIdx.x] = x0 ^ x1;
}

// HBM: one read and one write of 16 bytes per lane per step, grid-stride
__global__ void __launch_bounds__(PK_THREADS) peak_copy_kernel(uint4 *dst, const uint4 *src, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * PK_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * PK_THREADS)
        dst[i] = src[i];
}

template <class F>
hipError_t time_ms(F launch, int reps, float *ms)
{
    hipEvent_t a, b;
    hipError_t st = hipEventCreate(&a);
    if (st != hipSuccess) return st;
    if ((st = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return st;
    }
    launch();  // warm-up
    st = hipGetLastError();
    if (st == hipSuccess) st = hipEventRecord(a, nullptr);
    for (int i = 0; i < reps && st == hipSuccess; ++i) {
        launch();
        st = hipGetLastError();
    }
    if (st == hipSuccess) st = hipEventRecord(b, nullptr);
    if (st == hipSuccess) st = hipEventSynchronize(b);
    if (st == hipSuccess) st = hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st == hipSuccess) *ms /= (float)reps;
    return st;
}

}  // namespace
}  // namespace ea

extern "C" ea_status ea_measure_peaks(double *rates)
{
    using namespace ea;
    if (!rates) return EA_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return EA_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return EA_EDEVICE;
    const int blocks = cus * 8;  // eight four-wave workgroups per CU: eight waves per SIMD
    const size_t nout = (size_t)blocks * PK_THREADS;
    const size_t copy_bytes = (size_t)1 << 30;
    uint32_t *out = nullptr;
    uint4 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&out, nout * sizeof(uint32_t)) != hipSuccess) return EA_ENOMEM;
    if (hipMalloc(&src, copy_bytes) != hipSuccess || hipMalloc(&dst, copy_bytes) != hipSuccess) {
        (void)hipFree(out);
        if (src) (void)hipFree(src);
        return EA_ENOMEM;
    }
    const int rounds = 20000;
    const double lanes = (double)nout;
    const double valu_ops = lanes * rounds * PK_CHAINS;
    float ms = 0.f;
    hipError_t st = hipMemset(src, 0x5A, copy_bytes);
    const dim3 grid(blocks), block(PK_THREADS);
    if (st == hipSuccess)
        st = time_ms([&] { hipLaunchKernelGGL(peak_xor_kernel, grid, block, 0, nullptr, out, 1u, rounds); }, 3, &ms);
    if (st == hipSuccess) rates[0] = valu_ops / (ms * 1e-3);
    if (st == hipSuccess)
        st = time_ms([&] { hipLaunchKernelGGL(peak_mad64_kernel, grid, block, 0, nullptr, out, 1u, rounds); }, 3,
                     &ms);
    if (st == hipSuccess) rates[1] = valu_ops / (ms * 1e-3);
    if (st == hipSuccess)
        st = time_ms([&] { hipLaunchKernelGGL(peak_mulhi_kernel, grid, block, 0, nullptr, out, 1u, rounds); }, 3,
                     &ms);
    if (st == hipSuccess) rates[2] = valu_ops / (ms * 1e-3);
    const int lds_rounds = 4000;
    if (st == hipSuccess)
        st = time_ms([&] { hipLaunchKernelGGL(peak_lds_kernel, grid, block, 0, nullptr, out, 1u, lds_rounds); }, 3,
                     &ms);
    if (st == hipSuccess) rates[3] = lanes * lds_rounds * 8 * 16.0 / (ms * 1e-3);
    const size_t n16 = copy_bytes / 16;
    if (st == hipSuccess)
        st = time_ms([&] { hipLaunchKernelGGL(peak_copy_kernel, dim3(cus * 32), block, 0, nullptr, dst, src, n16); },
                     5, &ms);
    if (st == hipSuccess) rates[4] = 2.0 * (double)copy_bytes / (ms * 1e-3);
    if (st == hipSuccess)
        st = time_ms([&] { hipLaunchKernelGGL(peak_exp_kernel, grid, block, 0, nullptr, out, 1u, rounds); }, 3, &ms);
    if (st == hipSuccess) rates[5] = valu_ops / (ms * 1e-3);
    (void)hipFree(out);
    (void)hipFree(src);
    (void)hipFree(dst);
    return st == hipSuccess ? EA_OK : EA_EDEVICE;
}
