// adjoint.hpp -- pathwise gradients of the window mean velocity through the Euler-Maruyama or
// stochastic Heun map (Eqs. (1)-(3)), by a discrete adjoint with checkpointing and noise
// regeneration.
//
// Loss of set k: L_k = (1/N) sum_i J_i, J_i = (x_S - x_{S-W}) / (W dt), i.e. the mean drift
// velocity that abp_integrate reports for the same set (bit for bit). Gradient order:
// (U0, a, D, d2, q, c, gamma0, F0).
//
// Forward phase: each lane integrates its particle from the workload initial condition and stores
// its whole state (28 bytes) every K steps. Backward phase: for each segment [jK, (j+1)K) in
// reverse, the lane restores the checkpoint and recomputes the segment with regenerated Philox
// noise, leaving sub-checkpoints at absolute multiples of B steps (B = 16 by default, or 8; K is
// rounded up to a multiple of 16) in the workspace, or in LDS beside the noise when both fit
// (16-step staging). Then, for each sub-window in reverse, it restores the sub-checkpoint,
// recomputes the sub-window while staging the values the reverse step needs (cos and sin of the
// phase, v, e at every point where the drift is evaluated, and sigma*xi) in registers, and runs
// the adjoint recursion backwards over it. When the segment's noise fits in LDS (at most K steps
// x 64 lanes x 4 bytes per wavefront, for every four-wavefront block resident on a CU: one, or
// two for Euler-Maruyama ensembles of at least two wavefronts per SIMD), level 1 keeps each
// sigma*xi it draws there and the staged recomputation reads it back instead of running Philox
// and Box-Muller a second time. Euler-Maruyama keeps the K - B steps level 1 draws; Heun keeps
// the last sub-window's noise too (drawn by its staged recomputation), K steps in all, and its
// reverse steps read sigma*xi there instead of from registers. The recomputation reproduces the
// forward bits exactly (the integrator's state is resumable mid-span), so the result does not
// depend on K. Per-step gradient terms are summed in FP32 within each absolute B-step window and
// in FP64 across windows (that grouping does not depend on K either); tiles of 64 particles and
// sets are then reduced in a fixed order.
//
// The parameter table is a device array: each call first computes and checks every set's
// constants on the device (k_adj_rows), raising a status word in the workspace for a set that
// abp_integrate would reject (or with D <= 0, where the gradient w.r.t. D is undefined); the
// integration kernels then do nothing and the finalize writes NaN. The call only enqueues.
//
// Workspace layout (abp_adjoint_workspace_bytes):
//   AdjRow rows[n_sets] | i32 status | float ckpt[n_seg][7][N] | float sub[K/8][7][N] |
//   double loss_part[n_sets][tiles][2] | double grad_part[n_sets][tiles][8]
// (N = n_sets * tiles * 64 checkpoint slots: one per lane, also past a set's last particle)
//
// This header holds the kernels; adjoint_em.hip instantiates the 16-step Euler-Maruyama backward
// of the exact gradient, adjoint_fwd.hip the forward phase's look-ahead loop, adjoint.hip every
// other kernel and the host code (each source is built with the instruction schedule that
// measured faster for its kernels).
#pragma once

#include "reduce.hpp"

namespace abp {

// Per-set constants of the reverse step (derivatives of the drift), FP32.
struct RevCoef {
    float two_pi;      // 2 pi                (dU'/dU0 = 2 pi (c + 2a cos 2th))
    float four_pi_U0;  // 4 pi U0             (dU'/da  = 4 pi U0 cos 2th)
    float a2;          // 2a
    float eight_a;     // 8a                  (U'' = -4 pi^2 U0 sin th (1 + 8a cos th))
    float m4pi2U0_h;   // -4 pi^2 U0 dt/2     (the Heun corrector's weight on U'')
    float inv2D;       // 1 / (2D)            (d(sigma xi)/dD = sigma xi / (2D))
    // the Euler-Maruyama reverse step runs on Lam = dt lam, with the step's dt folded in here
    float m4pi2U0_dt;  // -4 pi^2 U0 dt
    float d2_dt, g0_dt, c_dt, m2d2_dt;  // d2 dt, gamma0 dt, c dt, -2 d2 dt
};

struct AdjRow {
    Coef k;
    RevCoef r;
    uint32_t pad[2];  // 96 bytes
};

struct AdjArgs {
    const AdjRow *rows;
    const int32_t *status;  // raised by k_adj_rows for an invalid set
    float *ckpt;        // [n_seg][7][N]
    float *sub;         // [K/8][7][N]
    double *loss_part;  // [n_sets][tiles][2]
    double *grad_part;  // [n_sets][tiles][8]
    const double *gloss;
    double *loss;
    double *grad;
    double *grad_particles;  // optional [n_sets][n][8]: dJ_i/dtheta per particle
    int64_t n;          // particles per set
    int64_t N;          // checkpoint slots (64 per tile)
    int64_t tiles;      // tiles per set
    int64_t S, W, K;    // steps, window, checkpoint interval
    double dt;
    uint32_t k0, k1;
    int32_t n_sets;
    float rho;        // per-step decay of the adjoint (1 = exact gradient)
    int32_t vform;    // 1: the loss enters as (1/W) sum of v_n over the window (used with rho < 1)
    int32_t z_slots;  // steps of noise each lane keeps in LDS (Heun K, Euler-Maruyama K - B)
    int32_t lds_wave;  // floats of LDS per wavefront (noise, then sub-checkpoints when SUBL)
};

constexpr int kAlign = 16;    // checkpoint intervals are multiples of this
constexpr int kMinStage = 8;  // the shortest staging window (sub-checkpoint slots: K / 8)
constexpr int kGrad = 8;      // gradient components: U0, a, D, d2, q, c, gamma0, F0

struct AdjLayout {
    size_t rows, status, ckpt, sub, loss, grad, total;
    int64_t n_seg, n_sub, tiles;
};

// Every lane of every wave (also lanes past a set's last particle) owns one slot in the
// checkpoint planes: N = n_sets * tiles * 64.
// Checkpoint interval actually used: the requested K (at most S: one segment) rounded up to a
// multiple of 16, so that every segment starts on a sub-window boundary of either scheme.
inline int64_t effective_K(int64_t K, int64_t S)
{
    K = K < S ? K : S;
    return (K + kAlign - 1) / kAlign * kAlign;
}

// Sizes are checked for overflow by the caller (layout_fits).
inline AdjLayout adj_layout(int32_t n_sets, int64_t n, int64_t S, int64_t K)
{
    AdjLayout L;
    K = effective_K(K, S);
    L.n_seg = (S + K - 1) / K;
    L.n_sub = K / kMinStage;
    L.tiles = (n + 63) / 64;
    const size_t N = (size_t)n_sets * (size_t)L.tiles * 64;
    L.rows = 0;
    L.status = align_up(sizeof(AdjRow) * (size_t)n_sets, 256);
    L.ckpt = align_up(L.status + sizeof(int32_t), 256);
    L.sub = align_up(L.ckpt + sizeof(float) * 7 * N * (size_t)L.n_seg, 256);
    L.loss = align_up(L.sub + sizeof(float) * 7 * N * (size_t)L.n_sub, 256);
    L.grad = align_up(L.loss + sizeof(double) * 2 * (size_t)n_sets * (size_t)L.tiles, 256);
    L.total = align_up(L.grad + sizeof(double) * kGrad * (size_t)n_sets * (size_t)L.tiles, 256);
    return L;
}

// Whole particle state in 7 planes of N floats (cell stored as its bit pattern).
__device__ __forceinline__ void put_state(float *base, int64_t N, int64_t g, const Particle &p)
{
    base[g] = __int_as_float(p.cell);
    base[N + g] = p.xf;
    base[2 * N + g] = p.v;
    base[3 * N + g] = p.e;
    base[4 * N + g] = p.lx;
    base[5 * N + g] = p.lv;
    base[6 * N + g] = p.le;
}

__device__ __forceinline__ Particle get_state(const float *base, int64_t N, int64_t g)
{
    Particle p;
    p.cell = __float_as_int(base[g]);
    p.xf = base[N + g];
    p.v = base[2 * N + g];
    p.e = base[3 * N + g];
    p.lx = base[4 * N + g];
    p.lv = base[5 * N + g];
    p.le = base[6 * N + g];
    return p;
}

// The lane's place: wave w of the grid covers tile (w mod tiles) of set (w / tiles). The wave
// index is taken from the first lane, so that set and tile are known to be wavefront-uniform
// (scalar registers, and scalar loads of the set's row).
struct Lane {
    int lane;
    int32_t set;
    int64_t tile, i, g;
    bool live;
};

__device__ __forceinline__ bool locate(const AdjArgs &a, Lane &L)
{
    L.lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane((uint32_t)threadIdx.x >> 6);
    if (wave >= (int64_t)a.n_sets * a.tiles)
        return false;  // wavefront-uniform
    L.set = (int32_t)(wave / a.tiles);
    L.tile = wave - (int64_t)L.set * a.tiles;
    L.i = L.tile * 64 + L.lane;
    L.live = L.i < a.n;
    L.g = wave * 64 + L.lane;
    return true;
}

__device__ __forceinline__ Particle initial_particle(uint32_t pid, uint32_t set, uint32_t k0,
                                                     uint32_t k1)
{
    const Philox4 r = philox4x32_10(0u, pid, set, kDomainInit, k0, k1);
    Particle p;
    p.cell = 0;
    p.xf = (float)(r.w[0] >> 8) * 0x1p-24f;
    p.v = p.e = 0.0f;
    p.lx = p.lv = p.le = 0.0f;
    return p;
}

// Forward phase: integrate, store a checkpoint at every multiple of K, reduce the loss.
template <int SCHEME, int LOOP>
__global__ __launch_bounds__(256) void k_adj_forward(AdjArgs a, const AdjRow *__restrict__ rows)
{
    Lane L;
    if (*a.status != ABP_OK || !locate(a, L))
        return;
    // the set's row by value (scalar registers): read once, whatever the kernel stores
    const AdjRow row = rows[L.set];
    const Stream s{a.k0, a.k1, (uint32_t)L.set};
    const uint32_t pid[1] = {(uint32_t)L.i};
    Particle p[1] = {initial_particle(pid[0], (uint32_t)L.set, a.k0, a.k1)};
    const int64_t wb = a.S - a.W;
    double xs[1] = {0.0}, xe[1];
    int64_t step = 0;
    for (int64_t j = 0; j * a.K < a.S; ++j) {
        put_state(a.ckpt + (size_t)j * 7 * a.N, a.N, L.g, p[0]);
        const int64_t end = (j + 1) * a.K < a.S ? (j + 1) * a.K : a.S;
        if (wb >= step && wb < end) {
            advance<SCHEME, 1, LOOP>(row.k, s, pid, p, step, wb);
            xs[0] = position64(p[0].cell, p[0].xf, p[0].lx);
        }
        advance<SCHEME, 1, LOOP>(row.k, s, pid, p, step, end);
    }
    if (wb == a.S)
        xs[0] = position64(p[0].cell, p[0].xf, p[0].lx);
    xe[0] = position64(p[0].cell, p[0].xf, p[0].lx);
    const bool live[1] = {L.live};
    reduce_tiles<1>(xe, xs, live, L.tile, a.n, L.lane, 0, a.loss_part + 2 * L.set * a.tiles,
                    nullptr);
}

// Values of one sub-window staged for the reverse sweep, per step: cos and sin of the phase
// 2 pi (x + phi), v and e (the rounded sums the drift saw), sigma xi; for Heun also cos, sin, v and
// e at the predictor point (the values the step's second drift saw).
// NB = steps per sub-window, 16 or 8. 16 halves the per-window overheads; for Euler-Maruyama 8
// stages half the registers, so that two wavefronts fit one SIMD at the kernel's natural size
// (the 16-step kernel has a build capped at 256 registers for that). The Heun kernel holds one
// wavefront per SIMD either way.
template <int SCHEME, int NB>
struct Stage;

template <int NB>
struct Stage<0, NB> {
    static constexpr int B = NB;
    float c[B], s[B], v[B], e[B], z[B];
};

template <int NB>
struct Stage<1, NB> {
    static constexpr int B = NB;
    float c[B], s[B], v[B], e[B], ct[B], st[B], vt[B], et[B], z[B];
};

// Recompute slot t of a sub-window (absolute step base + t), staging its inputs in the stage's
// slot ps. The noise is regenerated or (FROM_LDS) read from the lane's LDS copy zl[64 t] kept by
// level 1; regenerated noise is also kept there when zl is given. The staged predictor repeats
// step_heun's own expressions (the compiler merges the two), so it holds the values that step saw.
template <int SCHEME, bool FROM_LDS, class ST>
__device__ __forceinline__ void rec_slot(const Coef &k, const Stream &s, uint32_t pid, Particle &q,
                                         float &xb, Noise4 &z, int64_t base, int t, int ps, ST &B,
                                         float *zl, const float *zpre = nullptr)
{
    float zs;
    if constexpr (FROM_LDS) {
        zs = zpre ? zpre[t] : zl[64 * t];
    } else {
        if ((t & 3) == 0)
            z = noise_block((uint32_t)((base + t) >> 2), pid, s.set, s.k0, s.k1, k.bm);
        zs = z.z[t & 3];
        if (zl)
            zl[64 * t] = zs;
    }
    const float xc = xb + q.lx, vc = q.v + q.lv, ec = q.e + q.le;
    B.c[ps] = __builtin_amdgcn_cosf(xc);
    B.s[ps] = __builtin_amdgcn_sinf(xc);
    B.v[ps] = vc;
    B.e[ps] = ec;
    B.z[ps] = zs;
    if constexpr (SCHEME == 1) {
        const float xp = fmaf(vc, k.dt, xc);
        B.ct[ps] = __builtin_amdgcn_cosf(xp);
        B.st[ps] = __builtin_amdgcn_sinf(xp);
        float fv0, fe0;
        drift(k, xc, vc, ec, fv0, fe0);
        heun_predictor_ve(k, vc, ec, fv0, fe0, zs, B.vt[ps], B.et[ps]);
    }
    step<SCHEME>(k, q, xb, zs);
    if ((t & (kSpan - 1)) == kSpan - 1) {
        end_span(q);
        xb = q.xf + k.phi;
    }
}

// Level 1 over one whole sub-window starting at absolute step base: the same arithmetic as
// advance(), keeping each sigma*xi in the lane's LDS copy zw[64 t]. (Computing the next block's
// noise ahead here, as the forward can, measured slower in this register-heavy kernel.)
template <int SCHEME, int NB>
__device__ __forceinline__ void level1_window(const Coef &k, const Stream &s, uint32_t pid,
                                              Particle &p, int64_t base, float *zw)
{
#pragma unroll
    for (int b = 0; b < NB / kSpan; ++b) {
        const uint32_t blk = (uint32_t)(base >> 2) + 2 * b;
        const Noise4 z0 = noise_block(blk, pid, s.set, s.k0, s.k1, k.bm);
        const Noise4 z1 = noise_block(blk + 1, pid, s.set, s.k0, s.k1, k.bm);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            zw[64 * (kSpan * b + j)] = z0.z[j];
            zw[64 * (kSpan * b + 4 + j)] = z1.z[j];
        }
        span_steps<SCHEME>(k, p, z0, z1);
    }
}

// Adjoint state and the per-window FP32 sums the gradient is assembled from (Euler-Maruyama;
// Heun sums the same terms at both drift points with weights lam' and nu, and the factor dt/2 is
// applied at the end):
//   A0 = sum lam_v dt cos th      A1 = sum lam_v dt cos^2 th    A2 = sum lam_v sigma xi
//   A3 = sum lam_v dt e v         A4 = sum lam_e dt e v^2       A5 = sum lam_e dt
//   A6 = sum lam_e dt e           A7 = sum lam_v dt v           A8 = sum lam_v dt
// (lam = lambda_{n+1}); sum lam_v dt cos 2th = 2 A1 - A8 and the parameter constants are applied
// once at the end.
constexpr int kSums = 9;

struct Rev {
    float lx, lv, le;
    float A[kSums];
};

// Loss-side constants of the reverse sweep. wb = S - W. The exact form injects -1/(W dt) into
// lam_x at state index wb; the decayed form adds 1/W to lam_v at every window step n >= wb. Only
// the one sub-window holding step wb - 1 tests n per slot (CHECK); every other sub-window is
// entirely before or after the window start and takes the wavefront-uniform add_w instead.
struct RevCtx {
    int64_t wb;
    float jscale, invW, rho;
};

// Euler-Maruyama reverse step on Lam = dt lam (the loss-side constants in cx are scaled alike),
// lam_n = lam' + dt J(y)^T lam'.
template <int VFORM, bool CHECK, int NB>
__device__ __forceinline__ void rev_slot_em(const Coef &k, const RevCoef &rc,
                                            const Stage<0, NB> &B, int t, float z, int64_t n,
                                            const RevCtx &cx, float add_w, Rev &r)
{
    if (CHECK && !VFORM && n + 1 == cx.wb)
        r.lx -= cx.jscale;  // the window-start position enters J with weight -1/(W dt)
    const float c = B.c[t], sn = B.s[t], v = B.v[t], e = B.e[t];
    const float ev = e * v;
    const float lev = r.le * ev;
    const float wc = r.lv * c;
    r.A[0] += wc;
    r.A[1] = fmaf(wc, c, r.A[1]);
    r.A[2] = fmaf(r.lv, z, r.A[2]);
    r.A[3] = fmaf(r.lv, ev, r.A[3]);
    r.A[4] = fmaf(lev, v, r.A[4]);
    r.A[5] += r.le;
    r.A[6] = fmaf(r.le, e, r.A[6]);
    r.A[7] = fmaf(r.lv, v, r.A[7]);
    r.A[8] += r.lv;
    // transpose of the step Jacobian; U'' = -4 pi^2 U0 sin th (1 + 8a cos th)
    const float nlx = fmaf(-r.lv, rc.m4pi2U0_dt * (sn * fmaf(rc.eight_a, c, 1.0f)), r.lx);
    const float nlv =
        fmaf(rc.m2d2_dt, lev, fmaf(r.lx, k.dt, fmaf(r.lv, fmaf(rc.d2_dt, e, -rc.g0_dt), r.lv)));
    const float d2v = rc.d2_dt * v;
    const float nle = fmaf(r.lv, d2v, fmaf(-r.le, fmaf(d2v, v, rc.c_dt), r.le));
    if (VFORM) {
        r.lx = cx.rho * nlx;
        r.lv = fmaf(cx.rho, nlv, CHECK ? (n >= cx.wb ? cx.invW : 0.0f) : add_w);
        r.le = cx.rho * nle;
    } else {
        r.lx = nlx;
        r.lv = nlv;
        r.le = nle;
    }
}

// Reverse of one stochastic Heun step y' = y + dt/2 (f(y) + f(yp)) + sigma xi e_v with predictor
// yp = y + dt f(y) + sigma xi e_v, lam' = lam_{n+1}:
//   mu = J(yp)^T lam',  nu = lam' + dt mu,  lam_n = lam' + dt/2 (mu + J(y)^T nu);
// the parameter terms are dt/2 f_theta(yp)^T lam' + dt/2 f_theta(y)^T nu, and sigma enters
// through both the corrector and the predictor: (lam'_v + dt/2 mu_v) xi.
// J(y)^T w at a drift point with cos c, sin sn, v, e and ev = e v. The x component, -U''(x) w_v,
// is returned divided by 4 pi^2 U0 (the caller applies that constant together with the step's dt
// or dt/2, from the row), and we_ev = w_e e v, which the d2 term of the parameter sums shares.
__device__ __forceinline__ void jac_t(const Coef &k, const RevCoef &rc, float c, float sn, float v,
                                      float e, float ev, float wx, float wv, float we, float &ox,
                                      float &ov, float &oe, float &we_ev)
{
    ox = (sn * fmaf(rc.eight_a, c, 1.0f)) * wv;  // U''(x) w_v / (-4 pi^2 U0)
    const float d2v = k.d2 * v;
    we_ev = we * ev;
    ov = fmaf(-2.0f * k.d2, we_ev, fmaf(fmaf(k.d2, e, -k.g0), wv, wx));
    oe = fmaf(d2v, wv, -fmaf(d2v, v, k.c) * we);
}

__device__ __forceinline__ void add_terms(Rev &r, float c, float v, float e, float ev, float wv,
                                          float we, float we_ev)
{
    const float wc = wv * c;
    r.A[0] += wc;
    r.A[1] = fmaf(wc, c, r.A[1]);
    r.A[3] = fmaf(wv, ev, r.A[3]);
    r.A[4] = fmaf(we_ev, v, r.A[4]);
    r.A[5] += we;
    r.A[6] = fmaf(we, e, r.A[6]);
    r.A[7] = fmaf(wv, v, r.A[7]);
    r.A[8] += wv;
}

// PRED: the predictor's v and e come from the stage; otherwise they are recomputed here from the
// staged values by the forward's own expressions (the same bits, in fewer registers).
template <bool CHECK, bool PRED, int NB>
__device__ __forceinline__ void rev_slot_heun(const Coef &k, const RevCoef &rc,
                                              const Stage<1, NB> &B, int t, float z, int64_t n,
                                              const RevCtx &cx, Rev &r)
{
    if (CHECK && n + 1 == cx.wb)
        r.lx -= cx.jscale;
    const float h = k.half_dt;
    float vt, et;
    if constexpr (PRED) {
        vt = B.vt[t];
        et = B.et[t];
    } else {
        float fv0, fe0;
        drift_cos(k, B.c[t], B.v[t], B.e[t], fv0, fe0);
        heun_predictor_ve(k, B.v[t], B.e[t], fv0, fe0, z, vt, et);
    }
    const float evt = et * vt, ev = B.e[t] * B.v[t];
    float mx, mv, me, tp;
    jac_t(k, rc, B.ct[t], B.st[t], vt, et, evt, r.lx, r.lv, r.le, mx, mv, me, tp);
    // nu = lam' + dt mu (mu_x = 4 pi^2 U0 mx)
    const float nx = fmaf(-rc.m4pi2U0_dt, mx, r.lx), nv = fmaf(k.dt, mv, r.lv),
                ne = fmaf(k.dt, me, r.le);
    float px, pv, pe, ty;
    jac_t(k, rc, B.c[t], B.s[t], B.v[t], B.e[t], ev, nx, nv, ne, px, pv, pe, ty);
    add_terms(r, B.ct[t], vt, et, evt, r.lv, r.le, tp);  // times dt/2 at the end
    add_terms(r, B.c[t], B.v[t], B.e[t], ev, nv, ne, ty);
    r.A[2] = fmaf(fmaf(h, mv, r.lv), z, r.A[2]);
    r.lx = fmaf(-rc.m4pi2U0_h, mx + px, r.lx);
    r.lv = fmaf(h, mv + pv, r.lv);
    r.le = fmaf(h, me + pe, r.le);
}

// The step's sigma*xi comes from the stage, or (Heun with ZLDS) from the lane's LDS copy zr[64 t]
// of the window's noise, which then takes no registers in the stage; that lets the Heun
// predictor's v and e be staged (with 8-step windows they always are). The Euler-Maruyama kernel
// keeps its noise staged: it has the registers, and an LDS read in its short reverse step costs
// more than it saves.
// Slot t of a window (step base + t) is staged in slot ps of the stage (see slot_of).
template <int SCHEME, int VFORM, bool CHECK, bool ZLDS, class ST>
__device__ __forceinline__ void rev_slot(const Coef &k, const RevCoef &rc, const ST &B, int t,
                                         int ps, const float *zr, int64_t n, const RevCtx &cx,
                                         float add_w, Rev &r, const float *zpre = nullptr)
{
    const float z = (ZLDS && SCHEME == 1) ? (zpre ? zpre[t] : zr[64 * t]) : B.z[ps];
    if constexpr (SCHEME == 0)
        rev_slot_em<VFORM, CHECK>(k, rc, B, ps, z, n, cx, add_w, r);
    else
        rev_slot_heun<CHECK, ZLDS || ST::B == 8>(k, rc, B, ps, z, n, cx, r);
}

// One stage buffer serves the whole pipeline. A window is staged in order (slot t in stage slot
// t) or reversed (slot t in stage slot NB-1-t); while a trip reverses a window it recomputes the
// next one into the stage slots the reverse steps have just read, so the layout flips with every
// trip and the stage holds one window, not two.
template <bool REVERSED, int NB>
__device__ __forceinline__ constexpr int slot_of(int t)
{
    return REVERSED ? NB - 1 - t : t;
}

// Reverse the first `hi` slots of a staged sub-window starting at absolute step base, last first.
template <int SCHEME, int VFORM, bool CHECK, bool ZLDS, bool REVERSED, class ST>
__device__ __forceinline__ void rev_window(const Coef &k, const RevCoef &rc, const ST &B,
                                           const float *zr, int64_t base, int hi,
                                           const RevCtx &cx, float add_w, Rev &r)
{
#pragma unroll
    for (int t = ST::B - 1; t >= 0; --t)
        if (t < hi)
            rev_slot<SCHEME, VFORM, CHECK, ZLDS>(k, rc, B, t, slot_of<REVERSED, ST::B>(t), zr,
                                                 base + t, cx, add_w, r);
}

// Recompute the first `hi` slots of the sub-window starting at absolute step base from q,
// staging them into B.
template <int SCHEME, bool FROM_LDS, bool REVERSED, class ST>
__device__ __forceinline__ void rec_window(const Coef &k, const Stream &s, uint32_t pid,
                                           Particle &q, int64_t base, int hi, ST &B, float *zl)
{
    Noise4 z;
    float xb = q.xf + k.phi;
#pragma unroll
    for (int t = 0; t < ST::B; ++t)
        if (t < hi)
            rec_slot<SCHEME, FROM_LDS>(k, s, pid, q, xb, z, base, t,
                                       slot_of<REVERSED, ST::B>(t), B, zl);
}

// One pipeline trip: reverse window m, staged with layout REVERSED, while recomputing window m-1
// (from q) into the stage slots just read (so window m-1 comes out with the other layout). The
// sub-window holding the loss-window start (m == m_chk) runs the two halves one after the other.
// ZLDS: both windows' noise is in the lane's LDS copy (zr: window m, zl: window m-1).
template <int SCHEME, int VFORM, bool ZLDS, bool REVERSED, class ST>
__device__ __forceinline__ void trip(const Coef &k, const RevCoef &rc, const Stream &s,
                                     uint32_t pid, Particle &q, int64_t m, int64_t m_chk,
                                     const RevCtx &cx, ST &S, const float *zr, float *zl, Rev &r)
{
    constexpr int kB = ST::B;
    if (m == m_chk) {
        rev_window<SCHEME, VFORM, true, ZLDS, REVERSED>(k, rc, S, zr, m * kB, kB, cx, 0.0f, r);
        rec_window<SCHEME, ZLDS, !REVERSED>(k, s, pid, q, (m - 1) * kB, kB, S, zl);
        return;
    }
    const float add_w = (VFORM && m * kB >= cx.wb) ? cx.invW : 0.0f;
    Noise4 z;
    float xb = q.xf + k.phi;
    // ZLDS: both windows' noise is read from LDS into registers before the steps, so that no step
    // waits for an LDS read issued just before it (at one wavefront per SIMD nothing else hides
    // that latency)
    float zrec[kB], zrev[kB];
    if constexpr (ZLDS) {
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            zrec[t] = zl[64 * t];
            if constexpr (SCHEME == 1)
                zrev[t] = zr[64 * t];
        }
        // the values are used here, before the steps: the reads complete together
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            asm volatile("" ::"v"(zrec[t]));
            if constexpr (SCHEME == 1)
                asm volatile("" ::"v"(zrev[t]));
        }
    }
#pragma unroll
    for (int t = 0; t < kB; ++t) {
        // window m's slot u and window m-1's slot t share stage slot ps
        const int u = kB - 1 - t;
        const int ps = slot_of<REVERSED, kB>(u);
        rev_slot<SCHEME, VFORM, false, ZLDS>(k, rc, S, u, ps, zr, m * kB + u, cx, add_w, r,
                                             ZLDS ? zrev : nullptr);
        rec_slot<SCHEME, ZLDS>(k, s, pid, q, xb, z, (m - 1) * kB, t, ps, S, zl,
                               ZLDS ? zrec : nullptr);
    }
}

// Reverse a whole staged window with no recomputation beside it.
template <int SCHEME, int VFORM, bool ZLDS, bool REVERSED, class ST>
__device__ __forceinline__ void last_window(const Coef &k, const RevCoef &rc, int64_t m,
                                            int64_t m_chk, const RevCtx &cx, const ST &S,
                                            const float *zr, Rev &r)
{
    constexpr int kB = ST::B;
    if (m == m_chk) {
        rev_window<SCHEME, VFORM, true, ZLDS, REVERSED>(k, rc, S, zr, m * kB, kB, cx, 0.0f, r);
    } else {
        const float add_w = (VFORM && m * kB >= cx.wb) ? cx.invW : 0.0f;
        rev_window<SCHEME, VFORM, false, ZLDS, REVERSED>(k, rc, S, zr, m * kB, kB, cx, add_w, r);
    }
}

__device__ __forceinline__ void flush(Rev &r, double (&A64)[kSums])
{
#pragma unroll
    for (int i = 0; i < kSums; ++i) {
        A64[i] += (double)r.A[i];
        r.A[i] = 0.0f;
    }
}

// Backward phase. lam = dJ_i/dy_{n+1} while step n is reversed. VFORM selects the decayed
// estimator (see abp_adjoint_cfg.lookback; Euler-Maruyama only).
//
// Within a segment the sub-windows are processed as a software pipeline: while window m is
// reversed from the stage, window m-1 is recomputed into the stage slots already read, in the
// same instruction stream, so the two dependency chains fill each other's latency (the adjoint
// runs at one wavefront per SIMD for 2^16-particle ensembles).
//
// SUBL (with ZLDS): the segment's sub-checkpoints are kept in LDS too, after the noise, so that
// reading the next one costs an LDS read rather than an L2 round trip (the compiler parks the
// prefetched values in accumulation registers, which waits for them).
//
// OCC: wavefronts per SIMD the kernel is built for (2: at most 256 registers, for ensembles with
// at least two wavefronts per SIMD; 1: the registers the schedule wants, for the one-wavefront
// case).
//
// Each instance is 25-95 KB of code, more than the instruction cache holds, so where it starts
// matters: it is aligned to 8 KB, which pins its cache placement however the rest of the code
// object changes (identical code of the Heun kernel ran 1.6% slower after an unrelated change
// moved it; 8 KB alignment measured as fast as the best placement seen, 64 KB 2% slower).
template <int SCHEME, int VFORM, bool ZLDS, int NB, bool SUBL, int OCC>
__global__ __launch_bounds__(256, OCC) __attribute__((aligned(8192))) void
k_adj_backward(AdjArgs a, const AdjRow *__restrict__ rows)
{
    using ST = Stage<SCHEME, NB>;
    constexpr int kStage = NB;
    // ZLDS: per wavefront, [z_slots][64] floats of noise; SUBL: then [K/NB - 1][7][64] floats of
    // sub-checkpoints
    extern __shared__ float zbuf[];
    Lane L;
    if (*a.status != ABP_OK || !locate(a, L))
        return;
    // The set's row: through the restrict-qualified table (scalar loads where the constants are
    // used; the checkpoint stores cannot alias it), or, for the 8-step Euler-Maruyama kernel, which
    // has registers to spare, copied into registers once.
    AdjRow row_copy;
    const AdjRow *rp = rows + L.set;
    if constexpr (SCHEME == 0 && NB == 8) {
        row_copy = *rp;
        rp = &row_copy;
    }
    const AdjRow &row = *rp;
    const Coef &k = row.k;
    const RevCoef &rc = row.r;
    const Stream s{a.k0, a.k1, (uint32_t)L.set};
    const uint32_t pid[1] = {(uint32_t)L.i};
    const int64_t wb = a.S - a.W;
    RevCtx cx;
    cx.wb = wb;
    // Euler-Maruyama runs the reverse sweep on Lam = dt lam: its loss-side constants carry dt
    const double lam_scale = SCHEME == 0 ? a.dt : 1.0;
    cx.jscale = (float)(lam_scale / ((double)a.W * a.dt));
    cx.invW = (float)(lam_scale / (double)a.W);
    cx.rho = a.rho;
    const int64_t m_chk = wb >= 1 ? (wb - 1) / kStage : -1;  // sub-window holding step wb - 1
    // exact form: J = (x_S - x_{S-W}) / (W dt); decayed form: J = (1/W) sum_{n >= S-W} v_n, which
    // is the same function of the Euler-Maruyama path, with each v_n's sensitivity damped by rho
    // per step of look-back
    Rev r;
    r.lx = VFORM ? 0.0f : cx.jscale;
    r.lv = r.le = 0.0f;
#pragma unroll
    for (int i = 0; i < kSums; ++i)
        r.A[i] = 0.0f;
    double A64[kSums] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t N = a.N;
    // sub-checkpoint planes: in workspace memory (stride N, slot g) or in the wavefront's LDS
    // (stride 64, slot lane)
    float *sub = a.sub;
    int64_t sN = N, sg = L.g;
    float *const lds_wave = zbuf + (size_t)(threadIdx.x >> 6) * a.lds_wave;
    if constexpr (SUBL) {
        sub = lds_wave + (size_t)a.z_slots * 64;
        sN = 64;
        sg = L.lane;
    }

    const int64_t n_seg = (a.S + a.K - 1) / a.K;
    // Memory reads are issued one stage ahead of their use (the next segment's checkpoint while
    // the current segment is reversed, the next sub-checkpoint while the current sub-window is).
    Particle ck = get_state(a.ckpt + (size_t)(n_seg - 1) * 7 * N, N, L.g);
    for (int64_t j = n_seg - 1; j >= 0; --j) {
        const int64_t s0 = j * a.K;  // a multiple of kStage
        const int64_t s1 = s0 + a.K < a.S ? s0 + a.K : a.S;
        const int64_t m0 = s0 / kStage, m1 = (s1 - 1) / kStage;
        // level 1: recompute the segment up to its last sub-window, leaving a sub-checkpoint at
        // each earlier sub-window start; the last one's start state stays in registers
        Particle p[1] = {ck};
        int64_t step = s0;
        // ZLDS: the lane's LDS copy of the segment's noise, 64 floats apart per step from the start
        // of sub-window m0; zw(m) is sub-window m's part
        float *zl = nullptr;
        if constexpr (ZLDS)
            zl = lds_wave + L.lane;
        auto zw = [&](int64_t mm) { return ZLDS ? zl + (size_t)(mm - m0) * kStage * 64 : nullptr; };
        // the segment's last sub-window keeps the noise its staged recomputation draws only where
        // the reverse sweep reads it back (Heun)
        float *zlast = (ZLDS && SCHEME == 1) ? zw(m1) : nullptr;
        for (int64_t m = m0; m < m1; ++m) {
            put_state(sub + (size_t)(m - m0) * 7 * sN, sN, sg, p[0]);
            if constexpr (ZLDS)
                level1_window<SCHEME, NB>(k, s, pid[0], p[0], m * kStage, zw(m));
            else
                advance<SCHEME, 1, 1>(k, s, pid, p, step, (m + 1) * kStage);
        }
        if (j > 0)
            ck = get_state(a.ckpt + (size_t)(j - 1) * 7 * N, N, L.g);

        ST S;  // the stage (one window; see slot_of)
        Particle q = p[0];
        int64_t m = m1;
        const int hi1 = (int)(s1 - m1 * kStage);
        if (hi1 < kStage) {
            // the run's final sub-window is shorter: recompute and reverse it on its own
            rec_window<SCHEME, false, false>(k, s, pid[0], q, m1 * kStage, hi1, S, zlast);
            rev_window<SCHEME, VFORM, true, ZLDS, false>(k, rc, S, zw(m1), m1 * kStage, hi1, cx,
                                                        0.0f, r);
            flush(r, A64);
            if (m1 == m0)
                continue;
            m = m1 - 1;
            q = get_state(sub + (size_t)(m - m0) * 7 * sN, sN, sg);
        }
        // prologue: stage window m in order (the segment's last sub-window draws its noise here,
        // an earlier one has it in LDS already)
        if (ZLDS && m < m1)
            rec_window<SCHEME, true, false>(k, s, pid[0], q, m * kStage, kStage, S, zw(m));
        else
            rec_window<SCHEME, false, false>(k, s, pid[0], q, m * kStage, kStage, S, zlast);
        Particle nxt;
        if (m > m0)
            nxt = get_state(sub + (size_t)(m - 1 - m0) * 7 * sN, sN, sg);
        // steady state, two trips per loop pass: the stage's layout is in order at the top
        for (;;) {
            if (m == m0) {
                last_window<SCHEME, VFORM, ZLDS, false>(k, rc, m, m_chk, cx, S, zw(m), r);
                flush(r, A64);
                break;
            }
            q = nxt;
            if (m - 1 > m0)
                nxt = get_state(sub + (size_t)(m - 2 - m0) * 7 * sN, sN, sg);
            trip<SCHEME, VFORM, ZLDS, false>(k, rc, s, pid[0], q, m, m_chk, cx, S, zw(m),
                                             zw(m - 1), r);
            flush(r, A64);
            --m;
            if (m == m0) {
                last_window<SCHEME, VFORM, ZLDS, true>(k, rc, m, m_chk, cx, S, zw(m), r);
                flush(r, A64);
                break;
            }
            q = nxt;
            if (m - 1 > m0)
                nxt = get_state(sub + (size_t)(m - 2 - m0) * 7 * sN, sN, sg);
            trip<SCHEME, VFORM, ZLDS, true>(k, rc, s, pid[0], q, m, m_chk, cx, S, zw(m),
                                            zw(m - 1), r);
            flush(r, A64);
            --m;
        }
    }
    // dJ/d(U0, a, D, d2, q, c, gamma0, F0) from the sums (FP64); the Heun sums other than A2
    // carry their factor dt/2 here
    const double two_pi = 2.0 * 3.14159265358979323846;
    if constexpr (SCHEME == 1) {
#pragma unroll
        for (int i = 0; i < kSums; ++i)
            if (i != 2)
                A64[i] *= (double)k.half_dt;
    } else {
        A64[2] /= a.dt;  // sum of Lam_v sigma xi = dt sum lam_v sigma xi
    }
    const double cos2 = 2.0 * A64[1] - A64[8];  // sum of lam_v dt cos 2th
    double g[kGrad];
    g[0] = -two_pi * (A64[0] + (double)rc.a2 * cos2);
    g[1] = -(double)rc.four_pi_U0 * cos2;
    g[2] = (double)rc.inv2D * A64[2];
    g[3] = A64[3] - A64[4];
    g[4] = A64[5];
    g[5] = -A64[6];
    g[6] = -A64[7];
    g[7] = A64[8];
    if (a.grad_particles && L.live) {
        double *gp = a.grad_particles + kGrad * ((int64_t)L.set * a.n + L.i);
#pragma unroll
        for (int i = 0; i < kGrad; ++i)
            gp[i] = g[i];
    }
    // tile partials of the gradient components (lanes past the end hold zeros)
    if (L.tile * 64 < a.n) {
        double *gp = a.grad_part + kGrad * ((int64_t)L.set * a.tiles + L.tile);
#pragma unroll
        for (int i = 0; i < kGrad; ++i) {
            const double t = wave_sum(L.live ? g[i] : 0.0);
            if (L.lane == 0)
                gp[i] = t;
        }
    }
}

// Launch one backward variant: the LDS forms the host chose (ZLDS, and SUBL for 16-step staging).
template <int SCHEME, int VFORM, int NB, int OCC>
inline void launch_backward(bool zlds, bool subl, unsigned grid, size_t lds, hipStream_t st,
                            const AdjArgs &a)
{
    const dim3 g(grid), b(256);
    if constexpr (NB == 16) {
        if (subl) {
            hipLaunchKernelGGL((k_adj_backward<SCHEME, VFORM, true, NB, true, OCC>), g, b, lds, st,
                               a, a.rows);
            return;
        }
    }
    if (zlds)
        hipLaunchKernelGGL((k_adj_backward<SCHEME, VFORM, true, NB, false, OCC>), g, b, lds, st, a,
                           a.rows);
    else
        hipLaunchKernelGGL((k_adj_backward<SCHEME, VFORM, false, NB, false, OCC>), g, b, 0, st, a,
                           a.rows);
}

// The forward phase with the noise look-ahead loop (the small-ensemble form), defined in
// adjoint_fwd.hip.
void launch_forward_ahead(bool heun, unsigned grid, hipStream_t st, const AdjArgs &a);

// The 16-step Euler-Maruyama backward launches for the exact gradient, defined in adjoint_em.hip:
// wavefronts per SIMD occ (1, or 2 for the build capped at 256 registers).
void launch_backward_em16(int occ, bool zlds, bool subl, unsigned grid, size_t lds,
                          hipStream_t st, const AdjArgs &a);

}  // namespace abp
