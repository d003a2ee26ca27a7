// microbench.hip -- kernels that measure the memory and atomic peaks of the GPU the engine
// runs on, so that the transport kernels' rates can be stated as fractions of what the box
// itself sustains: a streaming copy (HBM bandwidth), random 4-byte gathers from tables of a
// chosen size (the voxel-gather pattern of Woodcock tracking, served by L2, the Infinity
// Cache or HBM depending on the size), and FP64 / int64 atomic adds spread over a table or
// concentrated on a few hot words (the image tally's pattern).  None of this is part of the
// transport; it only supplies peaks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "epidmc.h"

namespace {

constexpr int MB_WG = 256;

__global__ __launch_bounds__(MB_WG) void k_mb_copy(const uint4 *__restrict__ x, uint4 *__restrict__ y, size_t n)
{
    const size_t stride = (size_t)gridDim.x * MB_WG;
    for (size_t i = (size_t)blockIdx.x * MB_WG + threadIdx.x; i < n; i += stride) y[i] = x[i];
}

// Per thread a 32-bit linear congruential sequence; the index is its top `bits` bits (the
// well-mixed ones).  Addresses depend only on the sequence, so a thread keeps many loads in
// flight: this measures the gather throughput the memory system sustains.
__device__ __forceinline__ uint32_t lcg(uint32_t s) { return s * 1664525u + 1013904223u; }
__device__ __forceinline__ uint32_t seed_of() { return (blockIdx.x * MB_WG + threadIdx.x) * 2654435761u + 12345u; }

__global__ __launch_bounds__(MB_WG) void k_mb_gather(const uint32_t *t, int bits, uint32_t n_per,
                                                     uint32_t *sink)
{
    uint32_t s = seed_of(), acc = 0;
    const int sh = 32 - bits;
    for (uint32_t i = 0; i < n_per; ++i) {
        s = lcg(s);
        acc ^= t[s >> sh];
    }
    // stored only for one value, so the loads cannot be removed and almost nothing is written
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ __launch_bounds__(MB_WG) void k_mb_atomic_f64(double *t, int bits, uint32_t n_per)
{
    uint32_t s = seed_of();
    const int sh = 32 - bits;
    for (uint32_t i = 0; i < n_per; ++i) {
        s = lcg(s);
        atomicAdd(t + (s >> sh), 1.0);
    }
}

__global__ __launch_bounds__(MB_WG) void k_mb_atomic_u64(unsigned long long *t, int bits, uint32_t n_per)
{
    uint32_t s = seed_of();
    const int sh = 32 - bits;
    for (uint32_t i = 0; i < n_per; ++i) {
        s = lcg(s);
        atomicAdd(t + (s >> sh), 1ull);
    }
}

}  // namespace

extern "C" epidmc_status epidmc_microbench(int kind, void *dev_buf, size_t bytes, int log2_elems,
                                           uint32_t ops_per_thread, uint32_t threads, void *stream)
{
    if (!dev_buf || kind < 0 || kind > 3) return EPIDMC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (kind == 0) {
        const size_t n16 = bytes / 2 / 16;
        if (n16 == 0) return EPIDMC_E_SHAPE;
        const uint4 *x = (const uint4 *)dev_buf;
        uint4 *y = (uint4 *)dev_buf + n16;
        const unsigned grid = (unsigned)std::min<size_t>((n16 + MB_WG * 4 - 1) / (MB_WG * 4), 65536);
        hipLaunchKernelGGL(k_mb_copy, dim3(grid), dim3(MB_WG), 0, s, x, y, n16);
        return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
    }
    if (log2_elems < 1 || log2_elems > 31 || threads == 0 || threads % MB_WG || ops_per_thread == 0)
        return EPIDMC_E_ARG;
    const size_t elem = kind == 1 ? 4 : 8;
    if (((size_t)1 << log2_elems) * elem > bytes) return EPIDMC_E_WORKSPACE;
    const dim3 grid(threads / MB_WG);
    if (kind == 1)
        hipLaunchKernelGGL(k_mb_gather, grid, dim3(MB_WG), 0, s, (const uint32_t *)dev_buf, log2_elems, ops_per_thread,
                           (uint32_t *)dev_buf);
    else if (kind == 2)
        hipLaunchKernelGGL(k_mb_atomic_f64, grid, dim3(MB_WG), 0, s, (double *)dev_buf, log2_elems, ops_per_thread);
    else
        hipLaunchKernelGGL(k_mb_atomic_u64, grid, dim3(MB_WG), 0, s, (unsigned long long *)dev_buf, log2_elems,
                           ops_per_thread);
    return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
}
