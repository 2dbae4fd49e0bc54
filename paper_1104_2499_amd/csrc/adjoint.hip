// adjoint.hip -- the adjoint's host code (abp_adjoint, abp_adjoint_workspace_bytes), the
// per-set constants, the finalize kernel, and the kernel instances other than the 16-step
// Euler-Maruyama backward of the exact gradient and the forward phase's look-ahead loop (the
// method is described in adjoint.hpp).
#include "adjoint.hpp"

namespace abp {

// One block of kFinalizeThreads per set: loss = mean over particles of J_i (the same fixed-order
// combine as the plain integrator's); grad = gloss / N * sum of tiles, each component summed in
// the same fixed order.
__global__ __launch_bounds__(kFinalizeThreads) void k_adj_finalize(AdjArgs a, int32_t phase,
                                                                   int32_t *status)
{
    const int32_t k = blockIdx.x;
    const int tid = threadIdx.x;
    const int32_t st = *a.status;
    if (k == 0 && tid == 0 && status)
        *status = st;
    if (st != ABP_OK) {
        if (phase == 0 && tid == 0)
            a.loss[k] = __builtin_nan("");
        if (phase == 1 && tid < kGrad)
            a.grad[kGrad * (int64_t)k + tid] = __builtin_nan("");
        return;
    }
    if (phase == 0) {
        double o[2];
        finalize_set(a.loss_part + 2 * (int64_t)k * a.tiles, a.tiles, a.n, (double)a.W * a.dt, o);
        if (tid == 0)
            a.loss[k] = o[0];
        return;
    }
    __shared__ double red[kGrad][kFinalizeThreads / 64];
    const double *gp = a.grad_part + kGrad * (int64_t)k * a.tiles;
    double acc[kGrad];
#pragma unroll
    for (int r = 0; r < kGrad; ++r)
        acc[r] = 0.0;
    for (int64_t t = tid; t < a.tiles; t += kFinalizeThreads) {
#pragma unroll
        for (int r = 0; r < kGrad; ++r)
            acc[r] += gp[kGrad * t + r];
    }
#pragma unroll
    for (int r = 0; r < kGrad; ++r) {
        acc[r] = wave_sum(acc[r]);
        if ((tid & 63) == 0)
            red[r][tid >> 6] = acc[r];
    }
    __syncthreads();
    if (tid < kGrad) {
        double s = red[tid][0];
#pragma unroll
        for (int w = 1; w < kFinalizeThreads / 64; ++w)
            s += red[tid][w];
        a.grad[kGrad * (int64_t)k + tid] = s * (a.gloss[k] / (double)a.n);
    }
}

}  // namespace abp

using namespace abp;

// LDS limits of the current device: per block, and per CU (what the resident blocks share).
static size_t lds_attribute(hipDeviceAttribute_t which)
{
    int dev = 0, value = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&value, which, dev) != hipSuccess)
        return 0;
    return (size_t)value;
}

static size_t lds_per_block_limit()
{
    return lds_attribute(hipDeviceAttributeMaxSharedMemoryPerBlock);
}

static size_t lds_per_cu_limit()
{
    return lds_attribute(hipDeviceAttributeMaxSharedMemoryPerMultiprocessor);
}

// The checkpoint planes dominate the workspace: 28 bytes x lanes x segments, which can exceed
// 64-bit sizes for absurd inputs; such sizes are rejected.
static bool layout_fits(int32_t n_sets, int64_t n, int64_t S, int64_t K)
{
    const int64_t Ke = effective_K(K, S);
    const unsigned __int128 lanes = (unsigned __int128)n_sets * (unsigned __int128)((n + 63) / 64) * 64;
    const unsigned __int128 slots = (unsigned __int128)((S + Ke - 1) / Ke) + Ke / kMinStage;
    return lanes * slots * 28u < ((unsigned __int128)1 << 62);
}


extern "C" size_t abp_adjoint_workspace_bytes(int32_t n_sets, int64_t n_per_set, int64_t n_steps,
                                              int64_t ckpt_every)
{
    if (n_sets < 1 || n_per_set < 1 || n_steps < 1 || ckpt_every < 1 ||
        n_per_set > kMaxParticles / n_sets || n_steps > kMaxStepIndex ||
        !layout_fits(n_sets, n_per_set, n_steps, ckpt_every))
        return 0;
    return adj_layout(n_sets, n_per_set, n_steps, ckpt_every).total;
}

// Per-set constants of both phases, from the FP64 parameters (contraction off, as in make_coef).
__device__ __forceinline__ AdjRow make_adj_row(const abp_params &p, double dt)
{
#pragma clang fp contract(off)
    AdjRow r;
    r.k = make_coef(p, dt);
    r.r.two_pi = (float)(2.0 * kPi);
    r.r.four_pi_U0 = (float)(4.0 * kPi * p.U0);
    r.r.a2 = (float)(2.0 * p.a);
    r.r.eight_a = (float)(8.0 * p.a);
    r.r.m4pi2U0_h = (float)(-4.0 * kPi * kPi * p.U0 * (0.5 * dt));
    r.r.inv2D = (float)(1.0 / (2.0 * p.D));
    r.r.m4pi2U0_dt = (float)(-4.0 * kPi * kPi * p.U0 * dt);
    r.r.d2_dt = (float)(p.d2 * dt);
    r.r.g0_dt = (float)(p.gamma0 * dt);
    r.r.c_dt = (float)(p.c * dt);
    r.r.m2d2_dt = (float)(-2.0 * p.d2 * dt);
    r.pad[0] = r.pad[1] = 0u;
    return r;
}

// Every FP32 constant of the row is finite (a tiny D makes 1 / (2D) overflow, for instance).
__device__ __forceinline__ bool adj_row_ok(const AdjRow &r)
{
    const RevCoef &c = r.r;
    const float f[] = {c.two_pi, c.four_pi_U0, c.a2, c.eight_a, c.m4pi2U0_h, c.inv2D,
                       c.m4pi2U0_dt, c.d2_dt, c.g0_dt, c.c_dt, c.m2d2_dt};
    for (float x : f)
        if (!std::isfinite(x))
            return false;
    return coef_ok(r.k);
}

// One thread per set: the set's constants, and the status word raised (ABP_E_ARG) if they are
// invalid. The status word is cleared before this kernel runs.
__global__ __launch_bounds__(256) void k_adj_rows(int32_t n_sets, const abp_params *params,
                                                  double dt, AdjRow *rows, int32_t *status)
{
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n_sets)
        return;
    const abp_params p = params[k];
    const AdjRow r = make_adj_row(p, dt);
    if (!params_ok(p) || !(p.D > 0.0) || !adj_row_ok(r))
        atomicMax(status, (int32_t)ABP_E_ARG);
    rows[k] = r;
}

extern "C" abp_status abp_adjoint(int32_t phase, int32_t n_sets, const abp_params *d_params,
                                  int64_t n_per_set, const abp_adjoint_cfg *cfg, void *d_ws,
                                  size_t ws_bytes, double *d_loss, const double *d_gloss,
                                  double *d_grad, double *d_grad_particles, int32_t *d_status,
                                  void *stream)
{
    if ((phase != 0 && phase != 1) || !d_params || !aligned(d_params, 8) || !cfg || n_sets < 1 ||
        n_per_set < 1 || n_per_set > kMaxParticles / n_sets ||
        n_per_set > 0xFFFFFFFFll || !aligned(d_status, 4))
        return ABP_E_ARG;
    if (!(cfg->dt > 0.0) || !is_finite(cfg->dt) || cfg->n_steps < 1 ||
        cfg->n_steps > kMaxStepIndex || cfg->window < 1 || cfg->window > cfg->n_steps ||
        cfg->ckpt_every < 1 || cfg->lookback < 0 ||
        (cfg->scheme != ABP_EM && cfg->scheme != ABP_HEUN) ||
        (cfg->scheme == ABP_HEUN && cfg->lookback > 0) ||
        (cfg->stage_steps != 0 && cfg->stage_steps != 8 && cfg->stage_steps != 16))
        return ABP_E_ARG;
    if (!d_ws || !aligned(d_ws, 256))
        return ABP_E_ARG;
    if (phase == 0 && (!d_loss || !aligned(d_loss, 8)))
        return ABP_E_ARG;
    if (phase == 1 && (!d_gloss || !d_grad || !aligned(d_gloss, 8) || !aligned(d_grad, 8) ||
                       !aligned(d_grad_particles, 8)))
        return ABP_E_ARG;
    if (!layout_fits(n_sets, n_per_set, cfg->n_steps, cfg->ckpt_every))
        return ABP_E_ARG;
    const AdjLayout L = adj_layout(n_sets, n_per_set, cfg->n_steps, cfg->ckpt_every);
    if (ws_bytes < L.total)
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;

    hipStream_t st = as_stream(stream);
    char *ws = reinterpret_cast<char *>(d_ws);
    int32_t *status = reinterpret_cast<int32_t *>(ws + L.status);
    AdjRow *rows = reinterpret_cast<AdjRow *>(ws + L.rows);
    fill_u32(reinterpret_cast<uint32_t *>(status), 1, st);
    hipLaunchKernelGGL(k_adj_rows, dim3((unsigned)((n_sets + 255) / 256)), dim3(256), 0, st, n_sets,
                       d_params, cfg->dt, rows, status);
    if (hipGetLastError() != hipSuccess)
        return ABP_E_HIP;

    AdjArgs a{};
    a.rows = rows;
    a.status = status;
    a.ckpt = reinterpret_cast<float *>(ws + L.ckpt);
    a.sub = reinterpret_cast<float *>(ws + L.sub);
    a.loss_part = reinterpret_cast<double *>(ws + L.loss);
    a.grad_part = reinterpret_cast<double *>(ws + L.grad);
    a.gloss = d_gloss;
    a.loss = d_loss;
    a.grad = d_grad;
    a.grad_particles = phase == 1 ? d_grad_particles : nullptr;
    a.n = n_per_set;
    a.N = (int64_t)n_sets * L.tiles * 64;
    a.dt = cfg->dt;
    a.tiles = L.tiles;
    a.S = cfg->n_steps;
    a.W = cfg->window;
    a.K = effective_K(cfg->ckpt_every, cfg->n_steps);
    const Stream ks = make_stream(cfg->seed, 0);
    a.k0 = ks.k0;
    a.k1 = ks.k1;
    a.n_sets = n_sets;
    a.vform = cfg->lookback > 0 ? 1 : 0;
    a.rho = cfg->lookback > 0 ? (float)(1.0 - 1.0 / (double)cfg->lookback) : 1.0f;
    const int64_t waves = (int64_t)n_sets * L.tiles;
    const unsigned grid = (unsigned)((waves * 64 + 255) / 256);
    const bool heun = cfg->scheme == ABP_HEUN;
    if (phase == 0) {
        // the noise of the next block ahead of the steps when the grid holds at most two
        // wavefronts per SIMD (its own instruction stream is all a SIMD has), else in place
        const int cus = device_cus();
        const bool ahead = cus > 0 && waves <= (int64_t)cus * 4 * 2;
        if (ahead)
            launch_forward_ahead(heun, grid, st, a);
        else if (heun)
            hipLaunchKernelGGL((k_adj_forward<1, 1>), dim3(grid), dim3(256), 0, st, a, a.rows);
        else
            hipLaunchKernelGGL((k_adj_forward<0, 1>), dim3(grid), dim3(256), 0, st, a, a.rows);
    } else {
        // B = 16 is the default for both schemes. An Euler-Maruyama ensemble of at least two
        // wavefronts per SIMD runs two blocks per CU (whether or not the noise then fits in LDS:
        // the occupancy is worth more than the LDS copy): the 8-step kernel as it is, the 16-step
        // one through its build for 256 registers. Smaller ensembles, and the Heun backward, run
        // one wavefront per SIMD, with LDS sized for that one block.
        const int B = cfg->stage_steps == 8 ? 8 : 16;
        const int cus = device_cus();
        const bool two = !heun && cus > 0 && waves >= (int64_t)cus * 4 * 2;
        const int blocks_per_cu = two ? 2 : 1;
        a.z_slots = (int32_t)(heun ? a.K : a.K - B);
        // per 256-thread block (4 wavefronts): the noise, and with 16-step staging the
        // sub-checkpoints of one segment (all but its last sub-window)
        const size_t z_floats = (size_t)a.z_slots * 64;
        const size_t sub_floats = (size_t)(a.K / B - 1) * 7 * 64;
        // level-1 noise in LDS when every resident block's copy fits (and one block's share is
        // allowed); else it is regenerated
        const auto fits = [&](size_t bytes) {
            return bytes * blocks_per_cu <= lds_per_cu_limit() && bytes <= lds_per_block_limit();
        };
        const bool zlds = a.z_slots > 0 && fits(4 * sizeof(float) * z_floats);
        const bool subl = zlds && B == 16 && fits(4 * sizeof(float) * (z_floats + sub_floats));
        a.lds_wave = (int32_t)(z_floats + (subl ? sub_floats : 0));
        const size_t lds = zlds ? 4 * sizeof(float) * (size_t)a.lds_wave : 0;
        if (heun && B == 16)
            launch_backward<1, 0, 16, 1>(zlds, subl, grid, lds, st, a);
        else if (heun)
            launch_backward<1, 0, 8, 1>(zlds, subl, grid, lds, st, a);
        else if (B == 8 && a.vform)
            launch_backward<0, 1, 8, 1>(zlds, subl, grid, lds, st, a);
        else if (B == 8)
            launch_backward<0, 0, 8, 1>(zlds, subl, grid, lds, st, a);
        else if (a.vform && two)
            launch_backward<0, 1, 16, 2>(zlds, subl, grid, lds, st, a);
        else if (a.vform)
            launch_backward<0, 1, 16, 1>(zlds, subl, grid, lds, st, a);
        else
            launch_backward_em16(two ? 2 : 1, zlds, subl, grid, lds, st, a);
    }
    if (hipGetLastError() != hipSuccess)
        return ABP_E_HIP;
    hipLaunchKernelGGL(k_adj_finalize, dim3((unsigned)n_sets), dim3(kFinalizeThreads), 0, st, a,
                       phase, d_status);
    return launch_status();
}
