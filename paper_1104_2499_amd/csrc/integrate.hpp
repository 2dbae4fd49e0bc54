// integrate.hpp -- the single-set integrator kernel (Fig. 1's per-work-item loop, one particle per
// lane, with the fused window reduction) and its launch helpers. Each scheme's kernels are
// instantiated in a source file of their own (integrate_em.hip, integrate_heun.hip), so that each
// can be built with the compiler settings that suit its loop.
#pragma once

#include "reduce.hpp"

namespace abp {

// Device view of an abp_state: cell, xf, v, e and the low parts lo[0:n] = lx, lo[n:2n] = lv,
// lo[2n:3n] = le.
struct StateView {
    int32_t *cell;
    float *xf, *v, *e, *lo;
    int64_t n;

    __device__ __forceinline__ Particle load(int64_t i) const
    {
        Particle p;
        p.cell = cell[i];
        p.xf = xf[i];
        p.v = v[i];
        p.e = e[i];
        p.lx = lo[i];
        p.lv = lo[n + i];
        p.le = lo[2 * n + i];
        return p;
    }
    __device__ __forceinline__ void store(int64_t i, const Particle &p) const
    {
        cell[i] = p.cell;
        xf[i] = p.xf;
        v[i] = p.v;
        e[i] = p.e;
        lo[i] = p.lx;
        lo[n + i] = p.lv;
        lo[2 * n + i] = p.le;
    }
    __device__ __forceinline__ double x64(int64_t i) const
    {
        return position64(cell[i], xf[i], lo[i]);
    }
};

struct FwdArgs {
    StateView st;
    StateView snap;  // window snapshot (whole state); unused pointers may be null
    uint32_t id0;
    int32_t n_bins;
    Coef k;
    Stream s;
    int64_t step0, n_steps, win_begin;
    double *part;    // null: no reduction in this call
    uint32_t *hist;
    int64_t acc_stride;  // > 0: time-accumulated histogram every acc_stride absolute steps
    uint64_t *acc;       // [acc_bins]
    int32_t acc_bins;
};

constexpr size_t hist_offset(int64_t n)
{
    return align_up((size_t)n_tiles(n) * 2 * sizeof(double), 256);
}

// Advance the lane's particles to absolute step `stop`; with the time-accumulated histogram
// (COUNTED), stop after every absolute step that is a multiple of acc_stride and count x mod 1
// into loc.
template <int SCHEME, int PPL, int UNROLL, bool COUNTED>
__device__ __forceinline__ void advance_counted(const FwdArgs &a, const uint32_t (&pid)[PPL],
                                                Particle (&p)[PPL], const bool (&live)[PPL],
                                                int64_t &step, int64_t stop, uint32_t *loc)
{
    if constexpr (COUNTED) {
        for (int64_t nxt = (step / a.acc_stride + 1) * a.acc_stride; nxt <= stop;
             nxt += a.acc_stride) {
            advance<SCHEME, PPL, UNROLL>(a.k, a.s, pid, p, step, nxt);
#pragma unroll
            for (int q = 0; q < PPL; ++q)
                if (live[q])
                    atomicAdd(&loc[hist_bin(position64(p[q].cell, p[q].xf, p[q].lx),
                                            a.acc_bins)], 1u);
        }
    }
    advance<SCHEME, PPL, UNROLL>(a.k, a.s, pid, p, step, stop);
}

// Dynamic LDS of k_integrate: [acc_bins] u32 for the time-accumulated histogram (COUNTED), then
// [n_bins] u32 for the final-position histogram of a reducing call.
template <int SCHEME, int PPL, int UNROLL, bool COUNTED>
__global__ __launch_bounds__(256) void k_integrate(FwdArgs a)
{
    extern __shared__ uint32_t lds[];
    uint32_t *loc = lds;                                  // [acc_bins] when COUNTED
    uint32_t *hloc = lds + (COUNTED ? a.acc_bins : 0);    // [n_bins] when reducing
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t base = wave * 64 * PPL;
    const int64_t n = a.st.n;
    const bool hist = a.part && a.n_bins > 0;  // block-uniform
    // wavefront-uniform; with a block-level histogram every wave reaches the block barriers
    if (base >= n && !COUNTED && !hist)
        return;
    if constexpr (COUNTED)
        clear_hist(loc, a.acc_bins);
    if (hist)
        clear_hist(hloc, a.n_bins);

    if (base < n) {
        Particle p[PPL];
        uint32_t pid[PPL];
        bool live[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int64_t i = base + 64 * q + lane;
            live[q] = i < n;
            pid[q] = a.id0 + (uint32_t)i;
            if (live[q]) {
                p[q] = a.st.load(i);
            } else {
                p[q].cell = 0;
                p[q].xf = p[q].v = p[q].e = 0.0f;
                p[q].lx = p[q].lv = p[q].le = 0.0f;
            }
        }

        const int64_t end = a.step0 + a.n_steps;
        int64_t step = a.step0;
        double xs[PPL];
        const bool snap_here = a.win_begin >= a.step0 && a.win_begin <= end;
        if (snap_here) {
            advance_counted<SCHEME, PPL, UNROLL, COUNTED>(a, pid, p, live, step, a.win_begin, loc);
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                xs[q] = position64(p[q].cell, p[q].xf, p[q].lx);
                if (live[q])
                    a.snap.store(base + 64 * q + lane, p[q]);
            }
        }
        advance_counted<SCHEME, PPL, UNROLL, COUNTED>(a, pid, p, live, step, end, loc);

#pragma unroll
        for (int q = 0; q < PPL; ++q)
            if (live[q])
                a.st.store(base + 64 * q + lane, p[q]);

        if (a.part) {
            double xe[PPL];
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                xe[q] = position64(p[q].cell, p[q].xf, p[q].lx);
                if (!snap_here)
                    xs[q] = live[q] ? a.snap.x64(base + 64 * q + lane) : 0.0;
            }
            reduce_tiles<PPL>(xe, xs, live, base / 64, n, lane, a.n_bins, a.part, hloc);
        }
    }

    if constexpr (COUNTED) {
        __syncthreads();
        for (int b = threadIdx.x; b < a.acc_bins; b += blockDim.x)
            if (loc[b])
                atomicAdd(reinterpret_cast<unsigned long long *>(&a.acc[b]),
                          (unsigned long long)loc[b]);
    }
    if (hist)
        flush_hist(hloc, a.hist, a.n_bins);
}

template <int SCHEME, int PPL, int UNROLL, bool COUNTED = false>
inline void launch_integrate(const FwdArgs &a, int block, hipStream_t st)
{
    const int64_t waves = (a.st.n + 64 * PPL - 1) / (64 * PPL);
    const int64_t threads = waves * 64;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
    const size_t lds = sizeof(uint32_t) * ((COUNTED ? (size_t)a.acc_bins : 0) +
                                           (a.part ? (size_t)a.n_bins : 0));
    hipLaunchKernelGGL((k_integrate<SCHEME, PPL, UNROLL, COUNTED>), dim3(grid), dim3(block), lds,
                       st, a);
}

// The time-histogram variant runs one particle per lane and the in-place loop (its results, like
// every variant's, do not depend on the launch shape); only the block size is taken from tuning.
template <int SCHEME, int PPL>
inline void dispatch_loop(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    switch (sh.loop()) {
    case 1: launch_integrate<SCHEME, PPL, 1>(a, sh.block, st); break;
    case 2: launch_integrate<SCHEME, PPL, 2>(a, sh.block, st); break;
    default: launch_integrate<SCHEME, PPL, kAhead>(a, sh.block, st); break;
    }
}

template <int SCHEME>
inline void dispatch_integrate(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    if (a.acc_stride > 0)
        launch_integrate<SCHEME, 1, 1, true>(a, sh.block, st);
    else if (sh.ppl == 1)
        dispatch_loop<SCHEME, 1>(a, sh, st);
    else
        dispatch_loop<SCHEME, 2>(a, sh, st);
}

// Per-scheme entry points, defined in integrate_em.hip and integrate_heun.hip.
void dispatch_integrate_em(const FwdArgs &a, const Shape &sh, hipStream_t st);
void dispatch_integrate_heun(const FwdArgs &a, const Shape &sh, hipStream_t st);

}  // namespace abp
