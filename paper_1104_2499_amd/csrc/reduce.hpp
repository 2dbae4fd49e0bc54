// reduce.hpp -- ensemble reductions shared by the single-set and batched integrators.
//
// A set's particles are cut into 64-particle tiles (tile t = particles [64 t, 64 t + 64)). For each
// tile the lanes of one wavefront add the window displacement and its square in FP64 with a fixed
// butterfly; one wavefront later adds a set's tiles in a fixed order. The tiling does not depend
// on the launch shape, so every tuning gives the same bits, and a set gives the same bits alone
// or inside a sweep. Histogram counts are integer atomics (order-free).
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

// One wavefront: lane t adds tiles t, t + 64, ... in order, then the butterfly; lane 0 writes the
// mean drift velocity sum(delta) / (n window_time) and its standard error.
__device__ __forceinline__ void finalize_set(const double *part, int64_t ntiles, int64_t n,
                                             double window_time, double *out)
{
    const int lane = threadIdx.x & 63;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = lane; i < ntiles; i += 64) {
        s1 += part[2 * i];
        s2 += part[2 * i + 1];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
        const double mean_d = s1 / (double)n;
        double var_d = n > 1 ? (s2 - s1 * mean_d) / (double)(n - 1) : 0.0;
        if (var_d < 0.0)
            var_d = 0.0;
        out[0] = mean_d / window_time;
        out[1] = sqrt(var_d / (double)n) / window_time;
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t count);

// Zero `count` words with a kernel (not a memset node: safe inside captured graphs).
inline void fill_u32(uint32_t *p, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p,
                       count);
}

}  // namespace abp
