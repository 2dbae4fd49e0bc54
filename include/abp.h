/*
 * abp.h -- C ABI of libabp, an MI355X (gfx950) library for ensembles of active Brownian particles
 * with an energy depot on a periodic ratchet.
 *
 * Model (M. Zabicki, "OpenCL/OpenGL approach for studying active Brownian motion", Sec. 2):
 *   Eq. (1)  de/dt = q - c e - d2 e v^2
 *   Eq. (2)  dv/dt = F0 + d2 e v - gamma0 v - U'(x) + sqrt(2 D) xi(t),   dx/dt = v
 *   Eq. (3)  U(x)  = U0 [ sin 2pi(x + phi) + a sin 4pi(x + phi) ]
 * Each particle is one lane of a wavefront; its state stays in registers for the whole call, and
 * its Gaussian noise is regenerated in registers from a counter-based generator instead of being
 * read from memory (Sec. 2 prefers an on-device generator over host-filled random buffers).
 *
 * Noise contract. Philox4x32-10 (Salmon et al., SC'11) with key (seed mod 2^32, seed / 2^32) and
 * counter (n / 4, particle id, set id, 0) for absolute step n; the four words of one block become
 * four normals by Box-Muller (Fig. 1) on 23-bit uniforms u1 = 1 - (w0 >> 9) 2^-23 in (0, 1],
 * u2 = (w1 >> 9) 2^-23 in [0, 1): z0 = rho cos 2pi u2, z1 = rho sin 2pi u2, rho = sqrt(-2 ln u1),
 * and likewise (w2, w3) -> z2, z3. Step n uses z[n mod 4]. Initial positions: x0 = (w0 >> 8) 2^-24
 * of block (0, particle id, set id, 1); v0 = e0 = 0.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are HIP device memory owned by the caller; h_* are host memory; structs
 *    passed by pointer are host memory read during the call only. The library never frees or
 *    keeps caller memory after returning, allocates no device memory, and never prints.
 *  - Alignment: workspaces (d_ws) 256 bytes, which hipMalloc returns; FP64 and u64 arrays 8 bytes;
 *    FP32, int32 and u32 arrays 4 bytes. A misaligned pointer is ABP_E_ARG.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the null stream). The
 *    status is returned synchronously: arguments are validated before anything is enqueued, and
 *    on ABP_E_ARG / ABP_E_WORKSPACE / ABP_E_DEVICE nothing is written. ABP_E_HIP reports a
 *    launch error from the HIP runtime. Values that live in device tables (the batched sweep's
 *    and the adjoint's parameter tables) are checked on the device instead: the result is
 *    written to a device status word (d_status), and the outputs become NaN (see each call).
 *  - Results are deterministic: identical inputs give bit-identical outputs for every tuning and
 *    every repeat (FP64 partials are combined in a fixed order; histograms are integer counts).
 *  - Only gfx950 devices are accepted (ABP_E_DEVICE otherwise).
 *  - Every entry point only enqueues kernels (no host synchronisation, no copies, no memset),
 *    so any sequence of calls may be captured into a HIP graph once the first call on the
 *    device has run (that call caches the device check).
 */
#ifndef ABP_H
#define ABP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABP_ABI_VERSION 4

typedef enum abp_status {
    ABP_OK = 0,
    ABP_E_ARG = 1,       /* invalid argument (null/misaligned pointer, out-of-range value) */
    ABP_E_HIP = 2,       /* HIP runtime error while enqueuing */
    ABP_E_WORKSPACE = 3, /* workspace smaller than the matching *_workspace_bytes() query */
    ABP_E_DEVICE = 4     /* current device is not gfx950 */
} abp_status;

typedef enum abp_scheme { ABP_EM = 0, ABP_HEUN = 1 } abp_scheme;

/* Model parameters of Eqs. (1)-(3). D >= 0 (D = 0 is the deterministic limit). The kernels compute
 * in FP32: a call is rejected (ABP_E_ARG) unless every coefficient derived from the parameters and
 * the time step (2 pi U0, 8 pi U0 a, F0 + 4 pi U0 a, gamma0, d2, q, c, phi, dt, 2 D dt; for the
 * adjoint also 4 pi U0, 4 pi^2 U0 dt, 1 / (2D), ...) is finite in FP32 and dt is positive in FP32. */
typedef struct abp_params {
    double U0, a, phi, gamma0, F0, d2, q, c, D;
} abp_params;
#define ABP_N_PARAMS 9 /* a device parameter table is an array of rows of these 9 doubles */

/* One integration call. Step indices are absolute, so a run may be split into calls. */
typedef struct abp_run {
    double dt;          /* time step, > 0 */
    int64_t n_steps;    /* steps taken by this call, >= 0 */
    int64_t step0;      /* absolute index of the first step of this call, >= 0 */
    int64_t win_begin;  /* absolute time index at which the averaging window opens: the position
                           is copied into the snapshot before step win_begin is taken; -1 = none */
    uint64_t seed;      /* Philox key */
    uint32_t set_id;    /* Philox counter word 2 (parameter-set index) */
    int32_t scheme;     /* abp_scheme */
    /* Time-accumulated histogram of x mod 1 (the particle density the paper displays while the
     * ensemble runs, Sec. 2), single-set integrator only. hist_stride = 0: off. hist_stride > 0:
     * after every absolute step index n with step0 < n <= step0 + n_steps and n a multiple of
     * hist_stride, each particle's x_n mod 1 is counted into d_hist_acc[hist_bins] (bins as for
     * the final-position histogram). Counts are added to what d_hist_acc holds, so chunked calls
     * accumulate like one call; the caller zeroes it. hist_bins: power of two <= 4096. One call
 * takes at most 2^24 - 1 samples (n_steps / hist_stride < 2^24 - 1); chunk longer runs. */
    int64_t hist_stride;
    uint64_t *d_hist_acc;  /* device, 8-byte aligned */
    int32_t hist_bins;
    int32_t pad;
} abp_run;
/* step0 + n_steps must not exceed 2^34 (the block counter n/4 is one 32-bit word). */

/* Particle state in structure-of-arrays form, device memory. Sec. 2 of the paper asks single
 * precision to avoid adding very small numbers to very big ones; the state is therefore kept as
 * FP32 high/low pairs: x = cell + xf + lx with an integer cell, v = v + lv, e = e + le. The
 * integrator keeps xf in [-1/2, 1/2] (it moves the nearest integer into the cell every eight
 * steps, exactly while |xf| < 2^23; the initial state has xf in [0, 1)). d_lo holds 3n floats:
 * lx at [0, n), lv at [n, 2n), le at [2n, 3n). The low parts are part of the state (a run split
 * into calls is bit-identical to one call only if they are carried). Particle i has Philox id
 * id0 + i. */
typedef struct abp_state {
    int32_t *d_cell;  /* n */
    float *d_xf;      /* n */
    float *d_v;       /* n */
    float *d_e;       /* n */
    float *d_lo;      /* 3n */
    int64_t n;        /* >= 1, <= 2^31 */
    uint32_t id0;     /* id of particle 0; id0 + n - 1 must fit in 32 bits */
    uint32_t pad;
} abp_state;

/* Launch shape. Zero fields select the built-in default. block: threads per workgroup (64, 128
 * or 256); ppl: particles per lane (1 or 2); unroll: Philox blocks (4 steps each) per loop
 * iteration (1 or 2); waves_per_simd: residency target of the persistent batched launch (1-8);
 * lookahead: 1 = each block's noise right before its steps, 2 = the next block's noise computed
 * while the current block steps (needs unroll 1), 0 = automatic: 2 when the launch holds at most
 * two wavefronts per SIMD, else 1. No choice changes a bit of the results. */
typedef struct abp_tuning {
    int32_t block, ppl, unroll, waves_per_simd, lookahead;
} abp_tuning;

int abp_abi_version(void);
/* A static description of a status code; any int32 value is accepted ("unknown status" for
 * values that are no abp_status). */
const char *abp_status_str(int32_t status);

/* Initial condition of an ensemble: the state (x, v, e) of Eqs. (1)-(2) at t = 0 for every work
 * item of Fig. 1 (the paper does not fix it, Sec. 2; here x0 ~ U[0,1) on the 24-bit grid,
 * v0 = e0 = 0) for particles id0..id0+n-1 of set `set_id` under `seed` (see the noise contract).
 * Writes all of *s (low parts zeroed). */
abp_status abp_init_state(const abp_state *s, uint64_t seed, uint32_t set_id, void *stream);

/* Philox4x32-10 of m counters: d_ctr [m][4] u32, d_key [m][2] u32 -> d_out [m][4] u32. The
 * generator the integrators use, exposed so that it can be checked bit for bit. */
abp_status abp_philox(int64_t m, const uint32_t *d_ctr, const uint32_t *d_key, uint32_t *d_out,
                      void *stream);

/* Bytes of the reduction workspace for n particles and n_bins histogram bins (0 or a power of
 * two up to 4096): FP64 partial sums per 64-particle tile plus a u32 histogram. */
size_t abp_reduce_workspace_bytes(int64_t n, int32_t n_bins);

/* Advance the ensemble by r->n_steps steps of the chosen scheme (Eqs. (1)-(3); the per-step loop
 * of Fig. 1), in place on *s. Euler-Maruyama evaluates all drifts at the old state; Heun averages
 * the drifts at the old state and at the Euler predictor, with the same normal.
 *  snap: state copy written at time index win_begin when step0 <= win_begin <= step0+n_steps,
 *        and read (its position) when the window opened in an earlier call; may be NULL when
 *        neither happens.
 *  d_ws: if non-NULL, the call also reduces the ensemble at its end: per-tile FP64 sums of the
 *        window displacement and its square, and the histogram of x mod 1 (n_bins bins), are
 *        written to d_ws (ws_bytes >= abp_reduce_workspace_bytes(n, n_bins)); abp_reduce turns
 *        them into results. Requires a window (win_begin >= 0, win_begin <= step0 + n_steps).
 *  r->hist_stride > 0: the time-accumulated histogram is added to r->d_hist_acc as well.
 *  tune: NULL = default launch shape. */
abp_status abp_integrate(const abp_params *p, const abp_run *r, const abp_state *s,
                         const abp_state *snap, void *d_ws, size_t ws_bytes, int32_t n_bins,
                         const abp_tuning *tune, void *stream);

/* Finish a reduction left in d_ws by abp_integrate or abp_reduce_state for n particles, into the
 * ensemble quantities the paper computes from the trajectories (Sec. 2: the mean drift velocity
 * of the ratchet current, and the particle density over one period of the potential):
 * d_out[0] = mean drift velocity = sum(delta) / (n window_time), d_out[1] = its standard error,
 * d_hist[n_bins] = u64 counts of particles with floor(n_bins (x - floor x)) = b (clamped to
 * n_bins - 1), x = (cell + xf) + lx evaluated in FP64; delta is the same FP64 position at the end
 * minus that of the snapshot. d_hist may be NULL when n_bins = 0. ws_bytes must be at least
 * abp_reduce_workspace_bytes(n, n_bins) (ABP_E_WORKSPACE otherwise). */
abp_status abp_reduce(const void *d_ws, size_t ws_bytes, int64_t n, int32_t n_bins,
                      double window_time, double *d_out, uint64_t *d_hist, void *stream);

/* The reduction stage alone, from two states (window start and end): the ensemble averages of
 * Sec. 2 (mean drift velocity of the ratchet current from the window displacement of x in
 * Eq. (2), and the density of x over one period of the potential of Eq. (3)). Writes the same
 * partials into d_ws as abp_integrate does; abp_reduce finishes them. */
abp_status abp_reduce_state(const abp_state *snap, const abp_state *end, int32_t n_bins,
                            void *d_ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Allocation-free form of abp_integrate + abp_reduce, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * ------------------------------------------------------------------------------------------- */
#define ABP_NOALLOC_MAX_PARTICLES (1 << 24)

/* Writes exactly what abp_integrate(p, r, s, snap, ws, .., n_bins, tune) followed by
 * abp_reduce(ws, .., s->n, n_bins, window_time, d_out, d_hist) write (the state, the snapshot,
 * d_out[2], d_hist[n_bins]), bit for bit, but keeps the reduction partials in a fixed device
 * array of the library (4 MiB + 16 KiB per GPU, held until the process ends) instead of a caller
 * workspace. It calls no allocator. Requires a window (0 <= win_begin <= step0 + n_steps);
 * s->n > ABP_NOALLOC_MAX_PARTICLES returns ABP_E_WORKSPACE. Every call on a GPU shares that
 * GPU's array and clears what must start at zero: calls in order on one stream are safe, calls
 * that overlap in time on one GPU (different streams or host threads) race. */
abp_status abp_integrate_reduce_noalloc(const abp_params *p, const abp_run *r,
                                        const abp_state *s, const abp_state *snap,
                                        int32_t n_bins, double window_time, double *d_out,
                                        uint64_t *d_hist, const abp_tuning *tune, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Batched sweep: many parameter sets, each an ensemble of its own size and step count, in one
 * persistent launch (Sec. 2 runs one work item per parameter set concurrently).
 * ------------------------------------------------------------------------------------------- */
typedef struct abp_batch {
    double dt;        /* time step shared by all sets, > 0 */
    uint64_t seed;    /* Philox key shared by all sets; set k uses counter word 2 = k */
    int32_t scheme;   /* abp_scheme */
    int32_t n_bins;   /* histogram bins per set: 0 or a power of two up to 4096 */
} abp_batch;

/* Bytes of workspace for abp_integrate_batched with n_sets sets (1 <= n_sets <= 2^20) whose tile
 * counts ceil(n_traj[k] / 64) add up to n_tiles (or less: any upper bound of that sum will do,
 * n_sets <= n_tiles < 2^31); 0 if the sizes are invalid. */
size_t abp_batched_workspace_bytes(int32_t n_sets, int64_t n_tiles, int32_t n_bins);

/* Integrate n_sets independent ensembles and reduce each one, in one persistent launch. The tables
 * are device arrays read on the device: set k has parameters d_params[k] (rows of ABP_N_PARAMS
 * doubles), d_ntraj[k] >= 1 particles (ids 0..d_ntraj[k]-1, Philox set id k) started from the
 * workload initial condition, d_nsteps[k] in [1, 2^34] steps, and a window of the last
 * d_window[k] steps (1 <= window <= steps; d_window NULL = d_nsteps[k] / 2). Outputs:
 * d_out[2k], d_out[2k+1] = mean drift velocity and its standard error; d_hist[k n_bins + b] =
 * u64 histogram of the final x mod 1. Each set's results equal, bit for bit, those of
 * abp_init_state + abp_integrate + abp_reduce run on that set alone with set_id = k, for every
 * tuning. The work list (sets cut into tiles of 64 particles, longest step count first) is built
 * on the device in d_ws. The host validates the scalars, pointers and the per-set part of the
 * workspace; the device checks the tables: a set abp_integrate would reject is ABP_E_ARG, tiles
 * beyond the workspace's capacity ABP_E_WORKSPACE. Then nothing is integrated, d_out is set to
 * NaN and d_hist to zero. *d_status (a device int32; may be NULL) receives the device-side status
 * (ABP_OK when the sweep ran). The call only enqueues. tune: block, ppl, unroll and
 * waves_per_simd (grid = CUs x 4 x waves_per_simd waves); NULL = default. */
abp_status abp_integrate_batched(int32_t n_sets, const abp_params *d_params,
                                 const int32_t *d_ntraj, const int64_t *d_nsteps,
                                 const int64_t *d_window, const abp_batch *cfg,
                                 const abp_tuning *tune, void *d_ws, size_t ws_bytes,
                                 double *d_out, uint64_t *d_hist, int32_t *d_status,
                                 void *stream);

/* ---------------------------------------------------------------------------------------------
 * Pathwise gradient of the window mean velocity (the ratchet current of Sec. 2) with respect to
 * the parameters of Eqs. (1)-(3), through the Euler-Maruyama or stochastic Heun map of the
 * per-step loop of Fig. 1: a discrete adjoint with checkpoints every ckpt_every steps and Philox
 * noise regenerated in the backward pass.
 * ------------------------------------------------------------------------------------------- */
typedef struct abp_adjoint_cfg {
    double dt;           /* > 0 */
    int64_t n_steps;     /* S >= 1 */
    int64_t window;      /* W, 1 <= W <= S: the loss averages over the last W steps */
    int64_t ckpt_every;  /* K >= 1: forward checkpoint interval (e.g. about sqrt(S)); rounded up
                            to a multiple of 16 (see stage_steps). The gradient does not depend on
                            K (bit for bit) */
    uint64_t seed;       /* Philox key; set k uses counter word 2 = k */
    int64_t lookback;    /* 0: exact pathwise gradient. T > 0 (Euler-Maruyama only): each window
                            velocity's sensitivity is damped by (1 - 1/T) per step of look-back (a
                            biased, bounded-variance estimator for long chaotic horizons) */
    int32_t scheme;      /* ABP_EM or ABP_HEUN: the map whose discrete adjoint is taken */
    int32_t stage_steps; /* steps the backward pass stages in registers at a time: 0 = default
                            (16), or 8 or 16. For Euler-Maruyama ensembles of at least two
                            wavefronts per SIMD the backward runs two wavefronts per SIMD at
                            either length (16 is faster, with K <= 64 its sub-checkpoints stay in
                            LDS); the Heun backward runs one wavefront per SIMD either way and is
                            faster at 16. Changes the grouping of the FP32 gradient sums, not the
                            recursion */
} abp_adjoint_cfg;

/* Bytes of workspace: checkpoints (28 bytes per particle per segment), sub-checkpoints, and the
 * loss and gradient partials. 0 if the sizes are invalid. */
size_t abp_adjoint_workspace_bytes(int32_t n_sets, int64_t n_per_set, int64_t n_steps,
                                   int64_t ckpt_every);

/* phase 0 (forward): for each set k (parameters d_params[k], a device table of rows of
 * ABP_N_PARAMS doubles; n_per_set particles with ids 0..n-1 from the workload initial condition)
 * integrate S steps of cfg->scheme, store the checkpoints in d_ws, and write d_loss[k] = L_k =
 * (1/n) sum_i (x_S - x_{S-W}) / (W dt), the same value abp_integrate + abp_reduce give for that
 * set alone with set_id = k.
 * phase 1 (backward): with d_ws left by phase 0 for identical arguments, write
 * d_grad[8k + j] = d_gloss[k] * dL_k/dtheta_j, theta = (U0, a, D, d2, q, c, gamma0, F0), and,
 * if d_grad_particles is non-NULL, d_grad_particles[8 (k n + i) + j] = dJ_i/dtheta_j of particle
 * i of set k (unscaled; used for per-particle checks and gradient statistics).
 * The parameter table is checked on the device (each phase): a set abp_integrate would reject,
 * or one with D <= 0, makes the device-side status ABP_E_ARG; then nothing is integrated and
 * d_loss (phase 0) or d_grad (phase 1) is set to NaN. *d_status (a device int32; may be NULL)
 * receives that status. The call only enqueues. */
abp_status abp_adjoint(int32_t phase, int32_t n_sets, const abp_params *d_params,
                       int64_t n_per_set, const abp_adjoint_cfg *cfg, void *d_ws, size_t ws_bytes,
                       double *d_loss, const double *d_gloss, double *d_grad,
                       double *d_grad_particles, int32_t *d_status, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ABP_H */
