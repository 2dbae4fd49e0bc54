// reduce.hpp -- ensemble reductions shared by the single-set and batched integrators.
//
// A set's particles are cut into 64-particle tiles (tile t = particles [64 t, 64 t + 64)). For each
// tile the lanes of one wavefront add the window displacement and its square in FP64 with a fixed
// butterfly; one 256-thread block later adds a set's tiles in a fixed order (thread j takes tiles
// j, j + 256, ... in turn, then a butterfly per wavefront and the four wavefront sums in order).
// The tiling does not depend on the launch shape, so every tuning gives the same bits, and a set
// gives the same bits alone or inside a sweep. Histogram counts are integer atomics (order-free):
// the single-set kernels count into a per-block copy in LDS and add it to the global counts once
// per nonzero bin; the batched kernel, whose waves move between sets, counts into the set's global
// array directly.
#pragma once

#include "common.hpp"

namespace abp {

// Tile partials and histogram counts for the PPL particles of one lane; the lane's particle q
// belongs to local tile tile0 + q of a set of n particles. part and hist point at the set's own
// arrays. Lanes past the end contribute zero and count nothing.
template <int PPL>
__device__ __forceinline__ void reduce_tiles(const double (&xe)[PPL], const double (&xs)[PPL],
                                             const bool (&live)[PPL], int64_t tile0, int64_t n,
                                             int lane, int32_t n_bins, double *part,
                                             uint32_t *hist)
{
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        if ((tile0 + q) * 64 >= n)
            break;  // wavefront-uniform: this tile lies past the set's last particle
        const double d = live[q] ? xe[q] - xs[q] : 0.0;
        const double s1 = wave_sum(d);
        const double s2 = wave_sum(d * d);
        if (lane == 0) {
            part[2 * (tile0 + q)] = s1;
            part[2 * (tile0 + q) + 1] = s2;
        }
        if (n_bins > 0 && live[q])
            atomicAdd(&hist[hist_bin(xe[q], n_bins)], 1u);
    }
}

// Threads per block of every finalize kernel: the FP64 summation order depends on it.
constexpr int kFinalizeThreads = 256;

// One block of kFinalizeThreads threads: thread j adds tiles j, j + 256, ... in order, each
// wavefront adds its 64 sums by the butterfly, and thread 0 adds the four wavefront sums in order
// and writes the mean drift velocity sum(delta) / (n window_time) and its standard error.
__device__ __forceinline__ void finalize_set(const double *part, int64_t ntiles, int64_t n,
                                             double window_time, double *out)
{
    __shared__ double red[2][kFinalizeThreads / 64];
    const int tid = threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll 4
    for (int64_t i = tid; i < ntiles; i += kFinalizeThreads) {
        s1 += part[2 * i];
        s2 += part[2 * i + 1];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s1;
        red[1][tid >> 6] = s2;
    }
    __syncthreads();
    if (tid == 0) {
        s1 = red[0][0];
        s2 = red[1][0];
#pragma unroll
        for (int w = 1; w < kFinalizeThreads / 64; ++w) {
            s1 += red[0][w];
            s2 += red[1][w];
        }
        const double mean_d = s1 / (double)n;
        double var_d = n > 1 ? (s2 - s1 * mean_d) / (double)(n - 1) : 0.0;
        if (var_d < 0.0)
            var_d = 0.0;
        out[0] = mean_d / window_time;
        out[1] = sqrt(var_d / (double)n) / window_time;
    }
}

// Add a block's LDS histogram (n_bins u32 counts) to the global u32 counts, one atomic per
// nonzero bin. Every thread of the block calls it after the block's last count.
__device__ __forceinline__ void flush_hist(const uint32_t *loc, uint32_t *hist, int32_t n_bins)
{
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (loc[b])
            atomicAdd(&hist[b], loc[b]);
}

// Zero a block's LDS histogram; every thread of the block calls it before the block's first count.
__device__ __forceinline__ void clear_hist(uint32_t *loc, int32_t n_bins)
{
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        loc[b] = 0u;
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t count);

// Zero `count` words with a kernel (not a memset node: safe inside captured graphs).
inline void fill_u32(uint32_t *p, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p,
                       count);
}

}  // namespace abp
