// forward.hip -- the single-set entry points of the ensemble integrator (its kernel, Fig. 1's
// per-work-item loop with one particle per lane, is in integrate.hpp) and the reductions: window
// mean drift velocity and histogram of x mod 1.
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

#include "integrate.hpp"

namespace abp {

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
        r->n_steps > kMaxStepIndex || r->step0 > kMaxStepIndex - r->n_steps || r->win_begin < -1 ||
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
        dispatch_integrate_em(a, sh, st);
    else
        dispatch_integrate_heun(a, sh, st);
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
