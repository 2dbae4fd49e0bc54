// forward.hip -- the ensemble integrator (Fig. 1's per-work-item loop, one particle per lane) and
// its reductions: window mean drift velocity and histogram of x mod 1.
//
// Layout of the reduction workspace (abp_reduce_workspace_bytes):
//   double part[n_tiles][2]   sums of delta and delta^2 over each 64-particle tile, delta = window
//                             displacement in FP64; tile t = particles [64 t, 64 t + 64)
//   uint32 hist[n_bins]       counts of x mod 1 (integer atomics: order-free, hence deterministic);
//                             each block counts into LDS and adds its nonzero bins once at the end
// The optional time-accumulated histogram goes to a caller-owned u64 array instead, LDS-privatised
// in the same way.
// Tiles do not depend on the launch shape, and abp_reduce adds them in a fixed order, so the
// results are bit-identical for every tuning.
#include <mutex>

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

// Reduction from two stored states (window start, window end); one particle per lane, the
// histogram counted per block in LDS ([n_bins] u32 of dynamic LDS).
__global__ __launch_bounds__(256) void k_reduce_state(StateView snap, StateView end,
                                                      int32_t n_bins, double *part, uint32_t *hist)
{
    extern __shared__ uint32_t hloc[];
    const int lane = threadIdx.x & 63;
    const int64_t base = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64;
    const int64_t n = end.n;
    if (n_bins > 0)
        clear_hist(hloc, n_bins);
    if (base < n) {
        const int64_t i = base + lane;
        bool live[1] = {i < n};
        double xe[1] = {live[0] ? end.x64(i) : 0.0};
        double xs[1] = {live[0] ? snap.x64(i) : 0.0};
        reduce_tiles<1>(xe, xs, live, base / 64, n, lane, n_bins, part, hloc);
    }
    if (n_bins > 0)
        flush_hist(hloc, hist, n_bins);
}

// Fixed-order FP64 combine of the tile partials by one block of kFinalizeThreads (the same routine
// finishes each set of a batched sweep, so a set run alone and inside a sweep agree bit for bit).
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(const double *part, int64_t ntiles,
                                                               const uint32_t *hist32,
                                                               int32_t n_bins, int64_t n,
                                                               double window_time, double *out,
                                                               uint64_t *hist64)
{
    finalize_set(part, ntiles, n, window_time, out);
    for (int b = threadIdx.x; b < n_bins; b += kFinalizeThreads)
        hist64[b] = hist32[b];
}

template <int SCHEME, int PPL, int UNROLL, bool COUNTED = false>
static void launch_integrate(const FwdArgs &a, int block, hipStream_t st)
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
static void dispatch_loop(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    switch (sh.loop()) {
    case 1: launch_integrate<SCHEME, PPL, 1>(a, sh.block, st); break;
    case 2: launch_integrate<SCHEME, PPL, 2>(a, sh.block, st); break;
    default: launch_integrate<SCHEME, PPL, kAhead>(a, sh.block, st); break;
    }
}

template <int SCHEME>
static void dispatch_integrate(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    if (a.acc_stride > 0)
        launch_integrate<SCHEME, 1, 1, true>(a, sh.block, st);
    else if (sh.ppl == 1)
        dispatch_loop<SCHEME, 1>(a, sh, st);
    else
        dispatch_loop<SCHEME, 2>(a, sh, st);
}

constexpr Shape kDefaultForward = {256, 1, 1, 8, 0};

static void zero_hist(uint32_t *hist, int32_t n_bins, hipStream_t st)
{
    if (n_bins > 0)
        fill_u32(hist, n_bins, st);
}

}  // namespace abp

using namespace abp;

extern "C" size_t abp_reduce_workspace_bytes(int64_t n, int32_t n_bins)
{
    if (n < 1 || n > kMaxParticles || !bins_ok(n_bins))
        return 0;
    return hist_offset(n) + align_up((size_t)n_bins * sizeof(uint32_t), 256);
}

static StateView view(const abp_state *s)
{
    StateView v;
    v.cell = s->d_cell;
    v.xf = s->d_xf;
    v.v = s->d_v;
    v.e = s->d_e;
    v.lo = s->d_lo;
    v.n = s->n;
    return v;
}

// Validates an integration call and fills its kernel arguments, except the reduction outputs
// (a.part, a.hist), which the caller points at its workspace when `reduce` is set.
static abp_status plan_integrate(const abp_params *p, const abp_run *r, const abp_state *s,
                                 const abp_state *snap, bool reduce, int32_t n_bins,
                                 const abp_tuning *tune, FwdArgs &a, Shape &sh)
{
    if (!p || !r || !state_ok(s) || !params_ok(*p))
        return ABP_E_ARG;
    if (!(r->dt > 0.0) || !is_finite(r->dt) || !coef_ok(make_coef(*p, r->dt)) || r->n_steps < 0 ||
        r->step0 < 0 ||
        r->n_steps > kMaxStepIndex || r->step0 + r->n_steps > kMaxStepIndex || r->win_begin < -1 ||
        (r->scheme != ABP_EM && r->scheme != ABP_HEUN) || r->hist_stride < 0)
        return ABP_E_ARG;
    if (r->hist_stride > 0 && (r->hist_bins < 1 || !bins_ok(r->hist_bins) || !r->d_hist_acc ||
                               !aligned(r->d_hist_acc, 8)))
        return ABP_E_ARG;
    // a block's LDS counts are 32-bit: at most 2^32 - 1 samples of its (<= 256) particles per call
    if (r->hist_stride > 0 && (r->n_steps / r->hist_stride + 1) * 256 > (int64_t)0xFFFFFFFF)
        return ABP_E_ARG;
    const int64_t end = r->step0 + r->n_steps;
    const bool snap_write = r->win_begin >= r->step0 && r->win_begin <= end;
    if (reduce && (r->win_begin < 0 || r->win_begin > end))
        return ABP_E_ARG;  // a reduction needs a window that is open by the end of the call
    if ((snap_write || reduce) && (!state_ok(snap) || snap->n != s->n))
        return ABP_E_ARG;
    if (reduce && !bins_ok(n_bins))
        return ABP_E_ARG;
    if (!resolve_tuning(tune, kDefaultForward, sh))
        return ABP_E_ARG;
    resolve_lookahead(sh, (s->n + 64 * sh.ppl - 1) / (64 * sh.ppl));

    a = FwdArgs{};
    a.st = view(s);
    if (snap_write || reduce)
        a.snap = view(snap);
    a.id0 = s->id0;
    a.n_bins = reduce ? n_bins : 0;
    a.k = make_coef(*p, r->dt);
    a.s = make_stream(r->seed, r->set_id);
    a.step0 = r->step0;
    a.n_steps = r->n_steps;
    a.win_begin = r->win_begin;
    if (r->hist_stride > 0) {
        a.acc_stride = r->hist_stride;
        a.acc = r->d_hist_acc;
        a.acc_bins = r->hist_bins;
    }
    return ABP_OK;
}

// Enqueue the integration (and the zeroing of its histogram counts when it reduces).
static abp_status enqueue_integrate(const FwdArgs &a, const Shape &sh, int32_t scheme,
                                    hipStream_t st)
{
    if (a.part)
        zero_hist(a.hist, a.n_bins, st);
    if (scheme == ABP_EM)
        dispatch_integrate<0>(a, sh, st);
    else
        dispatch_integrate<1>(a, sh, st);
    return launch_status();
}

extern "C" abp_status abp_integrate(const abp_params *p, const abp_run *r, const abp_state *s,
                                    const abp_state *snap, void *d_ws, size_t ws_bytes,
                                    int32_t n_bins, const abp_tuning *tune, void *stream)
{
    const bool reduce = d_ws != nullptr;
    FwdArgs a;
    Shape sh;
    if (abp_status st = plan_integrate(p, r, s, snap, reduce, n_bins, tune, a, sh))
        return st;
    if (reduce && !aligned(d_ws, 256))
        return ABP_E_ARG;
    if (reduce && ws_bytes < abp_reduce_workspace_bytes(s->n, n_bins))
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;
    if (reduce) {
        a.part = reinterpret_cast<double *>(d_ws);
        a.hist = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(d_ws) + hist_offset(s->n));
    }
    return enqueue_integrate(a, sh, r->scheme, as_stream(stream));
}

extern "C" abp_status abp_reduce_state(const abp_state *snap, const abp_state *end,
                                       int32_t n_bins, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!state_ok(snap) || !state_ok(end) || snap->n != end->n || !bins_ok(n_bins) || !d_ws ||
        !aligned(d_ws, 256))
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
    hipLaunchKernelGGL(k_reduce_state, dim3(grid), dim3(256), sizeof(uint32_t) * (size_t)n_bins, st,
                       view(snap), view(end), n_bins, part, hist);
    return launch_status();
}

extern "C" abp_status abp_reduce(const void *d_ws, size_t ws_bytes, int64_t n, int32_t n_bins,
                                 double window_time, double *d_out, uint64_t *d_hist,
                                 void *stream)
{
    if (!d_ws || !aligned(d_ws, 256) || n < 1 || n > kMaxParticles || !bins_ok(n_bins) ||
        !(window_time > 0.0) || !is_finite(window_time) || !d_out || !aligned(d_out, 8) ||
        (n_bins > 0 && (!d_hist || !aligned(d_hist, 8))))
        return ABP_E_ARG;
    if (ws_bytes < abp_reduce_workspace_bytes(n, n_bins))
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;
    const double *part = reinterpret_cast<const double *>(d_ws);
    const uint32_t *hist = reinterpret_cast<const uint32_t *>(
        reinterpret_cast<const char *>(d_ws) + hist_offset(n));
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, as_stream(stream), part,
                       n_tiles(n), hist, n_bins, n, window_time, d_out, d_hist);
    return launch_status();
}

// ---------------------------------------------------------------------------------------------
// Allocation-free variant of abp_integrate + abp_reduce, for callers that cannot allocate device
// memory. The reduction workspace is a file-scope device array (one copy per GPU, held until the
// process ends), sized for kNoAllocMaxParticles particles and kMaxBins bins. Host code never
// passes the array's name to a kernel: it looks up the array's device address once per device
// (hipGetSymbolAddress, with that device current) and passes that pointer.
// ---------------------------------------------------------------------------------------------
namespace abp {

constexpr int64_t kNoAllocMaxParticles = ABP_NOALLOC_MAX_PARTICLES;
constexpr size_t kNoAllocScratchBytes =
    hist_offset(kNoAllocMaxParticles) + align_up((size_t)kMaxBins * sizeof(uint32_t), 256);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array, looked up on the first call per device.
static abp_status scratch_pointer(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return ABP_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return ABP_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ABP_OK;
}

}  // namespace abp

extern "C" abp_status abp_integrate_reduce_noalloc(const abp_params *p, const abp_run *r,
                                                   const abp_state *s, const abp_state *snap,
                                                   int32_t n_bins, double window_time,
                                                   double *d_out, uint64_t *d_hist,
                                                   const abp_tuning *tune, void *stream)
{
    FwdArgs a;
    Shape sh;
    if (abp_status st = plan_integrate(p, r, s, snap, true, n_bins, tune, a, sh))
        return st;
    if (!(window_time > 0.0) || !is_finite(window_time) || !d_out || !aligned(d_out, 8) ||
        (n_bins > 0 && (!d_hist || !aligned(d_hist, 8))))
        return ABP_E_ARG;
    if (s->n > kNoAllocMaxParticles)
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;
    void *ws = nullptr;
    if (abp_status st = scratch_pointer(&ws))
        return st;
    a.part = reinterpret_cast<double *>(ws);
    a.hist = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + hist_offset(s->n));
    hipStream_t st = as_stream(stream);
    if (abp_status e = enqueue_integrate(a, sh, r->scheme, st))
        return e;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, st, a.part, n_tiles(s->n),
                       a.hist, n_bins, s->n, window_time, d_out, d_hist);
    return launch_status();
}
