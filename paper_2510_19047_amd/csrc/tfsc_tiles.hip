// Per-tile maximum of the statistic over a bank (paper Sec. "Results", false-alarm
// probabilities: the background distribution is built from the largest statistic a
// noise-only search returns in each parameter tile, realisation by realisation).
//
// Three launches after a fill: the maximum per tile by an atomic maximum on the IEEE
// bit pattern (monotone for the non-negative values the statistic takes), the smallest
// index attaining it by an atomic minimum, and the mapping of empty tiles to index -1.
// Every pass is a plain kernel, so the sequence can be captured into a HIP graph.
#include "tfsc_kernels.hpp"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tfsc {

namespace {

constexpr unsigned long long kNoIndex = 0x7fffffffffffffffull;

__device__ __forceinline__ bool tile_entry(const double *stat, const int32_t *tile, int64_t i, int32_t n_tiles,
                                           int32_t &t, unsigned long long &bits) {
    const double v = stat[i];
    t = tile[i];
    if (t < 0 || t >= n_tiles || !(v >= 0.0)) return false;  // excluded: no tile, negative or NaN
    bits = (unsigned long long)__double_as_longlong(v + 0.0);  // -0 counts as +0
    return true;
}

__global__ void k_tile_fill(int32_t n_tiles, unsigned long long *mx, unsigned long long *arg) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) {
        mx[t] = 0ull;
        arg[t] = kNoIndex;
    }
}

__global__ void k_tile_max(const double *__restrict__ stat, const int32_t *__restrict__ tile, int64_t n,
                           int32_t n_tiles, unsigned long long *mx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t t;
        unsigned long long b;
        if (tile_entry(stat, tile, i, n_tiles, t, b)) atomicMax(mx + t, b);
    }
}

__global__ void k_tile_arg(const double *__restrict__ stat, const int32_t *__restrict__ tile, int64_t n,
                           int32_t n_tiles, const unsigned long long *__restrict__ mx, unsigned long long *arg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t t;
        unsigned long long b;
        if (tile_entry(stat, tile, i, n_tiles, t, b) && b == mx[t]) atomicMin(arg + t, (unsigned long long)i);
    }
}

__global__ void k_tile_finish(int32_t n_tiles, unsigned long long *mx, unsigned long long *arg) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles && arg[t] == kNoIndex) arg[t] = ~0ull;  // -1: the tile holds no template
}

}  // namespace

hipError_t launch_tile_max(const double *stat, const int32_t *tile, int64_t n, int32_t n_tiles, double *tile_max,
                           int64_t *tile_arg, hipStream_t st) {
    auto *mx = reinterpret_cast<unsigned long long *>(tile_max);
    auto *arg = reinterpret_cast<unsigned long long *>(tile_arg);
    const unsigned tb = (unsigned)((n_tiles + 255) / 256);
    hipLaunchKernelGGL(k_tile_fill, dim3(tb), dim3(256), 0, st, n_tiles, mx, arg);
    if (n > 0) {
        const int64_t want = (n + 255) / 256;
        const unsigned nb = (unsigned)(want < 4096 ? want : 4096);
        hipLaunchKernelGGL(k_tile_max, dim3(nb), dim3(256), 0, st, stat, tile, n, n_tiles, mx);
        hipLaunchKernelGGL(k_tile_arg, dim3(nb), dim3(256), 0, st, stat, tile, n, n_tiles, mx, arg);
    }
    hipLaunchKernelGGL(k_tile_finish, dim3(tb), dim3(256), 0, st, n_tiles, mx, arg);
    return hipGetLastError();
}

}  // namespace tfsc
