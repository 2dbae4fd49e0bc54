// abi_client.cpp -- a host program that drives libabp through its C ABI alone (include/abp.h and
// the HIP runtime's C API; no Python, no torch). It allocates the state, snapshot, reduction
// workspace and outputs with hipMalloc, runs the initial condition, one integration call with the
// window snapshot and fused reduction, and the finalize; then a three-set batched sweep whose
// parameter, trajectory, step and window tables it copies into device memory; then the adjoint's
// forward and backward phases for a two-set parameter table. It prints one JSON line with the
// results and the status of calls that must be rejected.
//
// usage: abi_client n steps window scheme(0 = EM, 1 = Heun) seed
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>

#include "abp.h"

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));     \
            std::exit(2);                                                              \
        }                                                                              \
    } while (0)

#define ABP_OK_OR_EXIT(call)                                                           \
    do {                                                                               \
        abp_status s_ = (call);                                                        \
        if (s_ != ABP_OK) {                                                            \
            std::fprintf(stderr, "%s failed: %s\n", #call, abp_status_str(s_));        \
            std::exit(3);                                                              \
        }                                                                              \
    } while (0)

static abp_state make_state(int64_t n)
{
    abp_state s = {};
    HIP_OK(hipMalloc((void **)&s.d_cell, sizeof(int32_t) * n));
    HIP_OK(hipMalloc((void **)&s.d_xf, sizeof(float) * n));
    HIP_OK(hipMalloc((void **)&s.d_v, sizeof(float) * n));
    HIP_OK(hipMalloc((void **)&s.d_e, sizeof(float) * n));
    HIP_OK(hipMalloc((void **)&s.d_lo, sizeof(float) * 3 * n));
    s.n = n;
    s.id0 = 0;
    return s;
}

static void free_state(abp_state &s)
{
    HIP_OK(hipFree(s.d_cell));
    HIP_OK(hipFree(s.d_xf));
    HIP_OK(hipFree(s.d_v));
    HIP_OK(hipFree(s.d_e));
    HIP_OK(hipFree(s.d_lo));
}

int main(int argc, char **argv)
{
    if (argc != 6) {
        std::fprintf(stderr, "usage: %s n steps window scheme seed\n", argv[0]);
        return 1;
    }
    const int64_t n = std::atoll(argv[1]);
    const int64_t steps = std::atoll(argv[2]);
    const int64_t window = std::atoll(argv[3]);
    const int32_t scheme = std::atoi(argv[4]);
    const uint64_t seed = std::strtoull(argv[5], nullptr, 10);
    const int32_t bins = 256;
    const double dt = 1e-3;

    HIP_OK(hipSetDevice(0));
    abp_state s = make_state(n), snap = make_state(n);
    const size_t ws_bytes = abp_reduce_workspace_bytes(n, bins);
    void *d_ws = nullptr;
    double *d_out = nullptr;
    uint64_t *d_hist = nullptr;
    HIP_OK(hipMalloc(&d_ws, ws_bytes));
    HIP_OK(hipMalloc((void **)&d_out, 2 * sizeof(double)));
    HIP_OK(hipMalloc((void **)&d_hist, bins * sizeof(uint64_t)));

    // the base ratchet: U0, a, phi, gamma0, F0, d2, q, c, D
    const abp_params p = {1.0, 0.25, 0.0, 1.0, 0.0, 1.0, 1.0, 0.1, 0.1};
    abp_run r = {};
    r.dt = dt;
    r.n_steps = steps;
    r.step0 = 0;
    r.win_begin = steps - window;
    r.seed = seed;
    r.set_id = 0;
    r.scheme = scheme;

    ABP_OK_OR_EXIT(abp_init_state(&s, seed, 0, nullptr));
    ABP_OK_OR_EXIT(abp_integrate(&p, &r, &s, &snap, d_ws, ws_bytes, bins, nullptr, nullptr));
    ABP_OK_OR_EXIT(abp_reduce(d_ws, ws_bytes, n, bins, (double)window * dt, d_out, d_hist, nullptr));

    double out[2];
    uint64_t hist[bins];
    HIP_OK(hipMemcpy(out, d_out, sizeof out, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hist, d_hist, sizeof hist, hipMemcpyDeviceToHost));
    uint64_t total = 0;
    for (int b = 0; b < bins; ++b)
        total += hist[b];

    // a negative step count is rejected before anything is enqueued
    abp_run bad = r;
    bad.n_steps = -1;
    const abp_status rejected = abp_integrate(&p, &bad, &s, &snap, d_ws, ws_bytes, bins, nullptr,
                                              nullptr);
    // so is a workspace one byte short
    const abp_status short_ws = abp_integrate(&p, &r, &s, &snap, d_ws, ws_bytes - 1, bins,
                                              nullptr, nullptr);

    // batched sweep over device tables: U0 varies, sizes are ragged
    const int32_t n_sets = 3;
    abp_params h_params[n_sets] = {p, p, p};
    h_params[1].U0 = 1.5;
    h_params[2].U0 = 0.7;
    const int32_t h_ntraj[n_sets] = {(int32_t)n, 100, 65};
    const int64_t h_nsteps[n_sets] = {steps, 500, 1001};
    const int64_t h_window[n_sets] = {window, 250, 400};
    int64_t tiles = 0;
    for (int k = 0; k < n_sets; ++k)
        tiles += (h_ntraj[k] + 63) / 64;
    const size_t bws_bytes = abp_batched_workspace_bytes(n_sets, tiles, bins);
    abp_params *d_params = nullptr;
    int32_t *d_ntraj = nullptr, *d_bstatus = nullptr;
    int64_t *d_nsteps = nullptr, *d_window = nullptr;
    void *d_bws = nullptr;
    double *d_bout = nullptr;
    uint64_t *d_bhist = nullptr;
    HIP_OK(hipMalloc((void **)&d_params, sizeof h_params));
    HIP_OK(hipMalloc((void **)&d_ntraj, sizeof h_ntraj));
    HIP_OK(hipMalloc((void **)&d_nsteps, sizeof h_nsteps));
    HIP_OK(hipMalloc((void **)&d_window, sizeof h_window));
    HIP_OK(hipMalloc((void **)&d_bstatus, sizeof(int32_t)));
    HIP_OK(hipMalloc(&d_bws, bws_bytes));
    HIP_OK(hipMalloc((void **)&d_bout, 2 * n_sets * sizeof(double)));
    HIP_OK(hipMalloc((void **)&d_bhist, (size_t)n_sets * bins * sizeof(uint64_t)));
    HIP_OK(hipMemcpy(d_params, h_params, sizeof h_params, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_ntraj, h_ntraj, sizeof h_ntraj, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_nsteps, h_nsteps, sizeof h_nsteps, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_window, h_window, sizeof h_window, hipMemcpyHostToDevice));
    abp_batch bcfg = {};
    bcfg.dt = dt;
    bcfg.seed = seed;
    bcfg.scheme = scheme;
    bcfg.n_bins = bins;
    ABP_OK_OR_EXIT(abp_integrate_batched(n_sets, d_params, d_ntraj, d_nsteps, d_window, &bcfg,
                                         nullptr, d_bws, bws_bytes, d_bout, d_bhist, d_bstatus,
                                         nullptr));
    double bout[2 * n_sets];
    int32_t bstatus = -1;
    HIP_OK(hipMemcpy(bout, d_bout, sizeof bout, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&bstatus, d_bstatus, sizeof bstatus, hipMemcpyDeviceToHost));
    // a workspace without room for one tile per set is refused on the host
    const abp_status short_bws = abp_integrate_batched(
        n_sets, d_params, d_ntraj, d_nsteps, d_window, &bcfg, nullptr, d_bws,
        abp_batched_workspace_bytes(n_sets, n_sets, bins) - 256, d_bout, d_bhist, d_bstatus,
        nullptr);

    // adjoint over a device parameter table: the base ratchet and U0 = 1.5, 700 particles each,
    // checkpoints every 100 steps; the backward phase weights the two losses by 1 and 1/2
    const int32_t a_sets = 2;
    const int64_t a_n = 700, a_ckpt = 100;
    abp_params h_ap[a_sets] = {p, p};
    h_ap[1].U0 = 1.5;
    const double h_gloss[a_sets] = {1.0, 0.5};
    abp_adjoint_cfg acfg = {};
    acfg.dt = dt;
    acfg.n_steps = steps;
    acfg.window = window;
    acfg.ckpt_every = a_ckpt;
    acfg.seed = seed;
    acfg.lookback = 0;
    acfg.scheme = scheme;
    acfg.stage_steps = 0;
    const size_t aws_bytes = abp_adjoint_workspace_bytes(a_sets, a_n, steps, a_ckpt);
    abp_params *d_ap = nullptr;
    void *d_aws = nullptr;
    double *d_loss = nullptr, *d_gloss = nullptr, *d_grad = nullptr;
    int32_t *d_astatus = nullptr;
    HIP_OK(hipMalloc((void **)&d_ap, sizeof h_ap));
    HIP_OK(hipMalloc(&d_aws, aws_bytes));
    HIP_OK(hipMalloc((void **)&d_loss, a_sets * sizeof(double)));
    HIP_OK(hipMalloc((void **)&d_gloss, sizeof h_gloss));
    HIP_OK(hipMalloc((void **)&d_grad, 8 * a_sets * sizeof(double)));
    HIP_OK(hipMalloc((void **)&d_astatus, sizeof(int32_t)));
    HIP_OK(hipMemcpy(d_ap, h_ap, sizeof h_ap, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_gloss, h_gloss, sizeof h_gloss, hipMemcpyHostToDevice));
    ABP_OK_OR_EXIT(abp_adjoint(0, a_sets, d_ap, a_n, &acfg, d_aws, aws_bytes, d_loss, nullptr,
                               nullptr, nullptr, d_astatus, nullptr));
    ABP_OK_OR_EXIT(abp_adjoint(1, a_sets, d_ap, a_n, &acfg, d_aws, aws_bytes, nullptr, d_gloss,
                               d_grad, nullptr, d_astatus, nullptr));
    double loss[a_sets], grad[8 * a_sets];
    int32_t astatus = -1;
    HIP_OK(hipMemcpy(loss, d_loss, sizeof loss, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(grad, d_grad, sizeof grad, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&astatus, d_astatus, sizeof astatus, hipMemcpyDeviceToHost));
    // a window longer than the run is rejected on the host
    abp_adjoint_cfg bad_a = acfg;
    bad_a.window = steps + 1;
    const abp_status adj_rejected = abp_adjoint(0, a_sets, d_ap, a_n, &bad_a, d_aws, aws_bytes,
                                                d_loss, nullptr, nullptr, nullptr, d_astatus,
                                                nullptr);

    std::printf("{\"abi_version\": %d, \"mean_v\": %.17g, \"stderr\": %.17g, \"hist_total\": %llu, "
                "\"hist_first\": %llu, \"rejected\": \"%s\", \"short_workspace\": \"%s\", "
                "\"sweep_status\": %d, \"sweep_mean_v\": [%.17g, %.17g, %.17g], "
                "\"sweep_stderr\": [%.17g, %.17g, %.17g], \"sweep_short_workspace\": \"%s\", "
                "\"adjoint_status\": %d, \"adjoint_loss\": [%.17g, %.17g], \"adjoint_grad\": [",
                abp_abi_version(), out[0], out[1], (unsigned long long)total,
                (unsigned long long)hist[0], abp_status_str(rejected), abp_status_str(short_ws),
                bstatus, bout[0], bout[2], bout[4], bout[1], bout[3], bout[5],
                abp_status_str(short_bws), astatus, loss[0], loss[1]);
    for (int j = 0; j < 8 * a_sets; ++j)
        std::printf("%s%.17g", j ? ", " : "", grad[j]);
    std::printf("], \"adjoint_rejected\": \"%s\"}\n", abp_status_str(adj_rejected));

    HIP_OK(hipFree(d_ap));
    HIP_OK(hipFree(d_aws));
    HIP_OK(hipFree(d_loss));
    HIP_OK(hipFree(d_gloss));
    HIP_OK(hipFree(d_grad));
    HIP_OK(hipFree(d_astatus));

    HIP_OK(hipFree(d_params));
    HIP_OK(hipFree(d_ntraj));
    HIP_OK(hipFree(d_nsteps));
    HIP_OK(hipFree(d_window));
    HIP_OK(hipFree(d_bstatus));
    HIP_OK(hipFree(d_bws));
    HIP_OK(hipFree(d_bout));
    HIP_OK(hipFree(d_bhist));

    HIP_OK(hipFree(d_ws));
    HIP_OK(hipFree(d_out));
    HIP_OK(hipFree(d_hist));
    free_state(s);
    free_state(snap);
    return 0;
}
