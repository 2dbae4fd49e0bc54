// forward.hip -- the ensemble integrator (Fig. 1's per-work-item loop, one particle per lane) and
// its reductions: window mean drift velocity and histogram of x mod 1.
//
// Layout of the reduction workspace (abp_reduce_workspace_bytes):
//   double part[n_tiles][2]   sums of delta and delta^2 over each 64-particle tile, delta = window
//                             displacement in FP64; tile t = particles [64 t, 64 t + 64)
//   uint32 hist[n_bins]       counts of x mod 1 (integer atomics: order-free, hence deterministic)
// Tiles do not depend on the launch shape, and abp_reduce adds them in a fixed order, so the
// results are bit-identical for every tuning.
#include "common.hpp"

namespace abp {

struct FwdArgs {
    int32_t *cell;
    float *xf, *v, *e;
    int32_t *scell;  // window snapshot (may be null when no window)
    float *sxf;
    int64_t n;
    uint32_t id0;
    int32_t n_bins;
    Coef k;
    Stream s;
    int64_t step0, n_steps, win_begin;
    double *part;    // null: no reduction in this call
    uint32_t *hist;
};

inline size_t hist_offset(int64_t n) { return align_up((size_t)n_tiles(n) * 2 * sizeof(double), 256); }

// Per-tile sums of the window displacement and the histogram update for the PPL particles held
// by one lane. Lanes past the end contribute zero and count nothing.
template <int PPL>
__device__ __forceinline__ void reduce_tiles(const Particle (&p)[PPL], const int32_t (&sc)[PPL],
                                             const float (&sx)[PPL], const bool (&live)[PPL],
                                             int64_t first_tile, int64_t n, int lane,
                                             int32_t n_bins, double *part, uint32_t *hist)
{
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        if ((first_tile + q) * 64 >= n)
            break;  // wavefront-uniform: this tile lies past the last particle
        double d = 0.0;
        if (live[q])
            d = (double)(p[q].cell - sc[q]) + ((double)p[q].xf - (double)sx[q]);
        const double s1 = wave_sum(d);
        const double s2 = wave_sum(d * d);
        if (lane == 0) {
            part[2 * (first_tile + q)] = s1;
            part[2 * (first_tile + q) + 1] = s2;
        }
        if (n_bins > 0 && live[q])
            atomicAdd(&hist[hist_bin(p[q].cell, p[q].xf, n_bins)], 1u);
    }
}

template <int SCHEME, int PPL, int UNROLL>
__global__ __launch_bounds__(256) void k_integrate(FwdArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t base = wave * 64 * PPL;
    if (base >= a.n)
        return;  // wavefront-uniform

    Particle p[PPL];
    uint32_t pid[PPL];
    bool live[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const int64_t i = base + 64 * q + lane;
        live[q] = i < a.n;
        pid[q] = a.id0 + (uint32_t)i;
        if (live[q]) {
            p[q].cell = a.cell[i];
            p[q].xf = a.xf[i];
            p[q].v = a.v[i];
            p[q].e = a.e[i];
        } else {
            p[q].cell = 0;
            p[q].xf = 0.0f;
            p[q].v = 0.0f;
            p[q].e = 0.0f;
        }
    }

    const int64_t end = a.step0 + a.n_steps;
    int64_t n = a.step0;
    int32_t sc[PPL];
    float sx[PPL];
    const bool snap_here = a.win_begin >= a.step0 && a.win_begin <= end;
    if (snap_here) {
        advance<SCHEME, PPL, UNROLL>(a.k, a.s, pid, p, n, a.win_begin);
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            sc[q] = p[q].cell;
            sx[q] = p[q].xf;
            if (live[q]) {
                const int64_t i = base + 64 * q + lane;
                a.scell[i] = sc[q];
                a.sxf[i] = sx[q];
            }
        }
    }
    advance<SCHEME, PPL, UNROLL>(a.k, a.s, pid, p, n, end);

#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        if (live[q]) {
            const int64_t i = base + 64 * q + lane;
            a.cell[i] = p[q].cell;
            a.xf[i] = p[q].xf;
            a.v[i] = p[q].v;
            a.e[i] = p[q].e;
        }
    }

    if (a.part) {
        if (!snap_here) {
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                const int64_t i = base + 64 * q + lane;
                sc[q] = live[q] ? a.scell[i] : 0;
                sx[q] = live[q] ? a.sxf[i] : 0.0f;
            }
        }
        reduce_tiles<PPL>(p, sc, sx, live, base / 64, a.n, lane, a.n_bins, a.part, a.hist);
    }
}

// Reduction from two stored states (window start, window end); one particle per lane.
__global__ __launch_bounds__(256) void k_reduce_state(const int32_t *scell, const float *sxf,
                                                      const int32_t *ecell, const float *exf,
                                                      int64_t n, int32_t n_bins, double *part,
                                                      uint32_t *hist)
{
    const int lane = threadIdx.x & 63;
    const int64_t base = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64;
    if (base >= n)
        return;
    const int64_t i = base + lane;
    Particle p[1];
    int32_t sc[1];
    float sx[1];
    bool live[1] = {i < n};
    p[0].cell = live[0] ? ecell[i] : 0;
    p[0].xf = live[0] ? exf[i] : 0.0f;
    p[0].v = p[0].e = 0.0f;
    sc[0] = live[0] ? scell[i] : 0;
    sx[0] = live[0] ? sxf[i] : 0.0f;
    reduce_tiles<1>(p, sc, sx, live, base / 64, n, lane, n_bins, part, hist);
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0u;
}

// Fixed-order FP64 combine of the tile partials: thread t adds tiles t, t + 1024, ... in order,
// then a fixed LDS tree. Also widens the u32 histogram to u64.
__global__ __launch_bounds__(1024) void k_finalize(const double *part, int64_t ntiles,
                                                   const uint32_t *hist32, int32_t n_bins,
                                                   int64_t n, double window_time, double *out,
                                                   uint64_t *hist64)
{
    __shared__ double s1s[1024];
    __shared__ double s2s[1024];
    const int t = threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = t; i < ntiles; i += 1024) {
        s1 += part[2 * i];
        s2 += part[2 * i + 1];
    }
    s1s[t] = s1;
    s2s[t] = s2;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            s1s[t] += s1s[t + w];
            s2s[t] += s2s[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double S1 = s1s[0], S2 = s2s[0];
        const double mean_d = S1 / (double)n;
        double var_d = n > 1 ? (S2 - S1 * mean_d) / (double)(n - 1) : 0.0;
        if (var_d < 0.0)
            var_d = 0.0;
        out[0] = mean_d / window_time;
        out[1] = sqrt(var_d / (double)n) / window_time;
    }
    for (int b = t; b < n_bins; b += 1024)
        hist64[b] = hist32[b];
}

template <int SCHEME, int PPL, int UNROLL>
static void launch_integrate(const FwdArgs &a, int block, hipStream_t st)
{
    const int64_t waves = (a.n + 64 * PPL - 1) / (64 * PPL);
    const int64_t threads = waves * 64;
    const unsigned grid = (unsigned)((threads + block - 1) / block);
    hipLaunchKernelGGL((k_integrate<SCHEME, PPL, UNROLL>), dim3(grid), dim3(block), 0, st, a);
}

template <int SCHEME>
static void dispatch_integrate(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    if (sh.ppl == 1) {
        if (sh.unroll == 1)
            launch_integrate<SCHEME, 1, 1>(a, sh.block, st);
        else
            launch_integrate<SCHEME, 1, 2>(a, sh.block, st);
    } else {
        if (sh.unroll == 1)
            launch_integrate<SCHEME, 2, 1>(a, sh.block, st);
        else
            launch_integrate<SCHEME, 2, 2>(a, sh.block, st);
    }
}

constexpr Shape kDefaultForward = {256, 1, 1, 8};

static void zero_hist(uint32_t *hist, int32_t n_bins, hipStream_t st)
{
    if (n_bins > 0)
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n_bins + 255) / 256)), dim3(256), 0, st,
                           hist, (int64_t)n_bins);
}

}  // namespace abp

using namespace abp;

extern "C" size_t abp_reduce_workspace_bytes(int64_t n, int32_t n_bins)
{
    if (n < 1 || n > kMaxParticles || !bins_ok(n_bins))
        return 0;
    return hist_offset(n) + align_up((size_t)n_bins * sizeof(uint32_t), 256);
}

extern "C" abp_status abp_integrate(const abp_params *p, const abp_run *r, const abp_state *s,
                                    const abp_state *snap, void *d_ws, size_t ws_bytes,
                                    int32_t n_bins, const abp_tuning *tune, void *stream)
{
    if (!p || !r || !state_ok(s) || !params_ok(*p))
        return ABP_E_ARG;
    if (!(r->dt > 0.0) || !is_finite(r->dt) || r->n_steps < 0 || r->step0 < 0 ||
        r->n_steps > kMaxStepIndex || r->step0 + r->n_steps > kMaxStepIndex || r->win_begin < -1 ||
        (r->scheme != ABP_EM && r->scheme != ABP_HEUN))
        return ABP_E_ARG;
    const int64_t end = r->step0 + r->n_steps;
    const bool snap_write = r->win_begin >= r->step0 && r->win_begin <= end;
    const bool reduce = d_ws != nullptr;
    if (reduce && (r->win_begin < 0 || r->win_begin > end))
        return ABP_E_ARG;  // a reduction needs a window that is open by the end of the call
    if ((snap_write || reduce) &&
        (!snap || !snap->d_cell || !snap->d_xf || !aligned(snap->d_cell, 4) ||
         !aligned(snap->d_xf, 4) || snap->n != s->n))
        return ABP_E_ARG;
    if (reduce && (!bins_ok(n_bins) || !aligned(d_ws, 256)))
        return ABP_E_ARG;
    Shape sh;
    if (!resolve_tuning(tune, kDefaultForward, sh))
        return ABP_E_ARG;
    if (reduce && ws_bytes < abp_reduce_workspace_bytes(s->n, n_bins))
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;

    FwdArgs a{};
    a.cell = s->d_cell;
    a.xf = s->d_xf;
    a.v = s->d_v;
    a.e = s->d_e;
    a.scell = (snap_write || reduce) ? snap->d_cell : nullptr;
    a.sxf = (snap_write || reduce) ? snap->d_xf : nullptr;
    a.n = s->n;
    a.id0 = s->id0;
    a.n_bins = reduce ? n_bins : 0;
    a.k = make_coef(*p, r->dt);
    a.s = make_stream(r->seed, r->set_id);
    a.step0 = r->step0;
    a.n_steps = r->n_steps;
    a.win_begin = r->win_begin;
    if (reduce) {
        a.part = reinterpret_cast<double *>(d_ws);
        a.hist = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(d_ws) + hist_offset(s->n));
    }
    hipStream_t st = as_stream(stream);
    if (reduce)
        zero_hist(a.hist, n_bins, st);
    if (r->scheme == ABP_EM)
        dispatch_integrate<0>(a, sh, st);
    else
        dispatch_integrate<1>(a, sh, st);
    return launch_status();
}

extern "C" abp_status abp_reduce_state(const abp_state *snap, const abp_state *end,
                                       int32_t n_bins, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!snap || !end || !snap->d_cell || !snap->d_xf || !end->d_cell || !end->d_xf ||
        !aligned(snap->d_cell, 4) || !aligned(snap->d_xf, 4) || !aligned(end->d_cell, 4) ||
        !aligned(end->d_xf, 4) || snap->n != end->n || end->n < 1 || end->n > kMaxParticles ||
        !bins_ok(n_bins) || !d_ws || !aligned(d_ws, 256))
        return ABP_E_ARG;
    if (ws_bytes < abp_reduce_workspace_bytes(end->n, n_bins))
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;
    hipStream_t st = as_stream(stream);
    double *part = reinterpret_cast<double *>(d_ws);
    uint32_t *hist = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(d_ws) +
                                                  hist_offset(end->n));
    zero_hist(hist, n_bins, st);
    const unsigned grid = (unsigned)((n_tiles(end->n) * 64 + 255) / 256);
    hipLaunchKernelGGL(k_reduce_state, dim3(grid), dim3(256), 0, st, snap->d_cell, snap->d_xf,
                       end->d_cell, end->d_xf, end->n, n_bins, part, hist);
    return launch_status();
}

extern "C" abp_status abp_reduce(const void *d_ws, int64_t n, int32_t n_bins, double window_time,
                                 double *d_out, uint64_t *d_hist, void *stream)
{
    if (!d_ws || !aligned(d_ws, 256) || n < 1 || n > kMaxParticles || !bins_ok(n_bins) ||
        !(window_time > 0.0) || !is_finite(window_time) || !d_out || !aligned(d_out, 8) ||
        (n_bins > 0 && (!d_hist || !aligned(d_hist, 8))))
        return ABP_E_ARG;
    if (abp_status st = check_device())
        return st;
    const double *part = reinterpret_cast<const double *>(d_ws);
    const uint32_t *hist = reinterpret_cast<const uint32_t *>(
        reinterpret_cast<const char *>(d_ws) + hist_offset(n));
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, as_stream(stream), part, n_tiles(n),
                       hist, n_bins, n, window_time, d_out, d_hist);
    return launch_status();
}
