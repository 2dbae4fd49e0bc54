/*
 * abp_oracle.c -- plain, slow FP64 CPU oracle for the active-Brownian-particle ensemble integrator.
 *
 * TEST INFRASTRUCTURE. This file is the reference the GPU library is checked against. Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg load it. It shares no code,
 * header, constant or helper with the HIP library; the two meet only through seeded inputs.
 *
 * What it computes (M. Zabicki, "OpenCL/OpenGL approach for studying active Brownian motion",
 * Sec. 2 and the pseudo-kernel of Fig. 1), one particle at a time, in IEEE double precision:
 *
 *   Eq. (1)  de/dt = q - c e - d2 e v^2                        (energy depot, coupling d2 = d)
 *   Eq. (2)  dv/dt = F0 + d2 e v - gamma0 v - U'(x) + sqrt(2D) xi(t)
 *            dx/dt = v
 *   Eq. (3)  U(x)  = U0 [ sin 2pi(x+phi) + a sin 4pi(x+phi) ]  (the paper's two-harmonic ratchet;
 *            its printed second harmonic reads 2pi, which cannot give a ratchet -- the 4pi reading
 *            and the (U0, a, phi) parametrisation are listed with the other readings in the docs)
 *
 * Fig. 1 runs, per work item, a loop of "draw uniform random numbers, Box-Muller them into
 * normals, update velocity and energy". Here the uniform generator is the counter-based
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11), keyed by the 64-bit seed, with counter (step/4, particle, set, domain); one Philox
 * block yields four normals, one per step. The update is Euler-Maruyama or stochastic Heun.
 *
 * Every function below is pinned by tests that do not re-type it (known-answer vectors and an
 * independent Philox implementation, closed forms, invariants, brute force, complex step).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct {
    double U0, a, phi, gamma0, F0, d2, q, c, D;
} orc_params;

enum { ORC_EM = 0, ORC_HEUN = 1 };
enum { DOMAIN_NOISE = 0, DOMAIN_INIT = 1 };

/* ---------------------------------------------------------------------------------------------
 * Philox4x32-10 (SC'11, Sec. 4): ten rounds of a multiply/xor Feistel-like bijection on four
 * 32-bit words; the two-word key is bumped by the Weyl constants between rounds.
 * ------------------------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t w0 = ctr[0], w1 = ctr[1], w2 = ctr[2], w3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)w0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)w2;
        uint32_t n0 = (uint32_t)(prod_b >> 32) ^ w1 ^ k0;
        uint32_t n1 = (uint32_t)prod_b;
        uint32_t n2 = (uint32_t)(prod_a >> 32) ^ w3 ^ k1;
        uint32_t n3 = (uint32_t)prod_a;
        w0 = n0; w1 = n1; w2 = n2; w3 = n3;
    }
    out[0] = w0; out[1] = w1; out[2] = w2; out[3] = w3;
}

void orc_philox_many(int64_t m, const uint32_t *ctrs, const uint32_t *keys, uint32_t *out)
{
    for (int64_t j = 0; j < m; ++j)
        orc_philox4x32_10(ctrs + 4 * j, keys + 2 * j, out + 4 * j);
}

static void philox_for(uint64_t seed, uint32_t blk, uint32_t pid, uint32_t set, uint32_t domain,
                       uint32_t r[4])
{
    uint32_t ctr[4] = {blk, pid, set, domain};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, r);
}

/* Box-Muller (the transformation named in Fig. 1): 23-bit uniforms u1 = 1 - (r >> 9) 2^-23 in
 * (0,1] and u2 = (r' >> 9) 2^-23 in [0,1), rho = sqrt(-2 ln u1), z = (rho cos 2pi u2,
 * rho sin 2pi u2). Words (r0,r1) give z0,z1 and (r2,r3) give z2,z3; step n of a particle uses
 * z[n mod 4] of block n/4. */
static void normals4(uint64_t seed, uint32_t pid, uint32_t set, uint32_t blk, double z[4])
{
    uint32_t r[4];
    philox_for(seed, blk, pid, set, DOMAIN_NOISE, r);
    for (int pair = 0; pair < 2; ++pair) {
        double u1 = 1.0 - (double)(r[2 * pair] >> 9) * 0x1p-23;
        double u2 = (double)(r[2 * pair + 1] >> 9) * 0x1p-23;
        double rho = sqrt(-2.0 * log(u1));
        z[2 * pair] = rho * cos(2.0 * ORC_PI * u2);
        z[2 * pair + 1] = rho * sin(2.0 * ORC_PI * u2);
    }
}

void orc_normals(uint64_t seed, uint32_t pid, uint32_t set, int64_t step0, int64_t count, double *z)
{
    double blk[4];
    for (int64_t j = 0; j < count; ++j) {
        int64_t n = step0 + j;
        if (j == 0 || n % 4 == 0)
            normals4(seed, pid, set, (uint32_t)(n / 4), blk);
        z[j] = blk[n % 4];
    }
}

/* Initial condition of the workloads: x0 ~ U[0,1) from the 24 high bits of the first word of
 * Philox block (0, particle, set, 1); v0 = e0 = 0. */
void orc_init_state(int64_t n, uint64_t seed, uint32_t set, const uint32_t *ids, double *x,
                    double *v, double *e)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t pid = ids ? ids[i] : (uint32_t)i;
        uint32_t r[4];
        philox_for(seed, 0u, pid, set, DOMAIN_INIT, r);
        x[i] = (double)(r[0] >> 8) * 0x1p-24;
        v[i] = 0.0;
        e[i] = 0.0;
    }
}

/* Ratchet potential and its derivatives, Eq. (3) in the two-harmonic form. */
double orc_potential(const orc_params *p, double x)
{
    double th = 2.0 * ORC_PI * (x + p->phi);
    return p->U0 * (sin(th) + p->a * sin(2.0 * th));
}

static double dU(const orc_params *p, double x)
{
    double th = 2.0 * ORC_PI * (x + p->phi);
    return 2.0 * ORC_PI * p->U0 * (cos(th) + 2.0 * p->a * cos(2.0 * th));
}

static double d2U(const orc_params *p, double x)
{
    double th = 2.0 * ORC_PI * (x + p->phi);
    return -4.0 * ORC_PI * ORC_PI * p->U0 * (sin(th) + 4.0 * p->a * sin(2.0 * th));
}

/* Right-hand side of Eqs. (1)-(2) without the noise term. */
static void drift(const orc_params *p, double x, double v, double e, double f[3])
{
    f[0] = v;
    f[1] = p->F0 - p->gamma0 * v + p->d2 * e * v - dU(p, x);
    f[2] = p->q - p->c * e - p->d2 * e * v * v;
}

/* One step of the scheme. EM evaluates every drift at the old state; Heun (the stochastic
 * trapezoid / improved Euler for additive noise) averages the drift at the old state and at the
 * EM predictor, reusing the same normal. */
static void one_step(const orc_params *p, int scheme, double dt, double sig, double z, double y[3])
{
    double f[3], pred[3];
    drift(p, y[0], y[1], y[2], f);
    pred[0] = y[0] + f[0] * dt;
    pred[1] = y[1] + f[1] * dt + sig * z;
    pred[2] = y[2] + f[2] * dt;
    if (scheme == ORC_EM) {
        memcpy(y, pred, sizeof pred);
        return;
    }
    double g[3];
    drift(p, pred[0], pred[1], pred[2], g);
    y[0] = y[0] + 0.5 * (f[0] + g[0]) * dt;
    y[1] = y[1] + 0.5 * (f[1] + g[1]) * dt + sig * z;
    y[2] = y[2] + 0.5 * (f[2] + g[2]) * dt;
}

/* Sensitivity model of single-precision state rounding (not part of the method): after each step
 * x moves by eps*u0 (absolute: a position fraction in [0,1) carries absolute rounding), and v, e
 * are scaled by (1 + eps*u1), (1 + eps*u2), with u uniform on [-1,1) from Philox domain 3. With
 * eps = 2^-24 it measures how far the dynamics itself amplifies FP32-sized rounding. */
static void perturb(uint64_t seed, uint32_t pid, uint32_t set, int64_t step, double eps, double y[3])
{
    uint32_t r[4];
    philox_for(seed, (uint32_t)step, pid, set, 3u, r);
    double u[3];
    for (int j = 0; j < 3; ++j)
        u[j] = (double)(r[j] >> 8) * 0x1p-23 - 1.0;
    y[0] += eps * u[0];
    y[1] *= 1.0 + eps * u[1];
    y[2] *= 1.0 + eps * u[2];
}

/* Advance n particles from absolute step step0 by n_steps steps (Fig. 1's loop).
 * x_snap[i] receives x at absolute time index win_begin when step0 <= win_begin <= step0+n_steps
 * (i.e. before step win_begin is taken); v_sum[i] (optional) accumulates v_n over the steps with
 * n >= win_begin, the time-average estimator of the mean velocity. eps != 0 applies the rounding
 * sensitivity model after every step. Returns 0, or -1 on bad input. */
int orc_integrate(const orc_params *p, int scheme, double dt, int64_t step0, int64_t n_steps,
                  int64_t win_begin, uint64_t seed, uint32_t set, int64_t n, const uint32_t *ids,
                  double *x, double *v, double *e, double *x_snap, double *v_sum, double eps)
{
    if (!(dt > 0.0) || n_steps < 0 || step0 < 0 || n < 0 || p->D < 0.0)
        return -1;
    if (n_steps > 0 && (step0 + n_steps - 1) / 4 > 0xFFFFFFFFll)
        return -1; /* the last step's noise block must fit the 32-bit counter word */
    const double sig = sqrt(2.0 * p->D * dt);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t pid = ids ? ids[i] : (uint32_t)i;
        double y[3] = {x[i], v[i], e[i]};
        double z[4];
        double vs = v_sum ? v_sum[i] : 0.0;
        for (int64_t k = 0; k < n_steps; ++k) {
            int64_t step = step0 + k;
            if (step == win_begin && x_snap)
                x_snap[i] = y[0];
            if (k == 0 || step % 4 == 0)
                normals4(seed, pid, set, (uint32_t)(step / 4), z);
            if (win_begin >= 0 && step >= win_begin)
                vs += y[1];
            one_step(p, scheme, dt, sig, z[step % 4], y);
            if (eps != 0.0)
                perturb(seed, pid, set, step, eps, y);
        }
        if (win_begin == step0 + n_steps && x_snap)
            x_snap[i] = y[0];
        x[i] = y[0];
        v[i] = y[1];
        e[i] = y[2];
        if (v_sum)
            v_sum[i] = vs;
    }
    return 0;
}

/* Ensemble outputs: mean drift velocity from the displacement over the window (summed in
 * particle order), its standard error, and the histogram of x mod 1 in n_bins equal bins. */
void orc_reduce(int64_t n, const double *x_snap, const double *x_end, double window_time,
                int32_t n_bins, double out[2], uint64_t *hist)
{
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = x_end[i] - x_snap[i];
        s1 += d;
        s2 += d * d;
    }
    double mean_d = s1 / (double)n;
    double var_d = n > 1 ? (s2 - s1 * mean_d) / (double)(n - 1) : 0.0;
    if (var_d < 0.0)
        var_d = 0.0;
    out[0] = mean_d / window_time;
    out[1] = sqrt(var_d / (double)n) / window_time;
    if (hist && n_bins > 0) {
        for (int32_t b = 0; b < n_bins; ++b)
            hist[b] = 0;
        for (int64_t i = 0; i < n; ++i) {
            double frac = x_end[i] - floor(x_end[i]);
            int64_t b = (int64_t)floor(frac * (double)n_bins);
            if (b >= n_bins)
                b = n_bins - 1;
            hist[b] += 1;
        }
    }
}

/* Classical fourth-order Runge-Kutta on the deterministic part of Eqs. (1)-(2) (D ignored). */
void orc_rk4(const orc_params *p, double dt, int64_t n_steps, int64_t n, double *x, double *v,
             double *e)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double y[3] = {x[i], v[i], e[i]};
        for (int64_t k = 0; k < n_steps; ++k) {
            double k1[3], k2[3], k3[3], k4[3], t[3];
            drift(p, y[0], y[1], y[2], k1);
            for (int j = 0; j < 3; ++j) t[j] = y[j] + 0.5 * dt * k1[j];
            drift(p, t[0], t[1], t[2], k2);
            for (int j = 0; j < 3; ++j) t[j] = y[j] + 0.5 * dt * k2[j];
            drift(p, t[0], t[1], t[2], k3);
            for (int j = 0; j < 3; ++j) t[j] = y[j] + dt * k3[j];
            drift(p, t[0], t[1], t[2], k4);
            for (int j = 0; j < 3; ++j)
                y[j] += dt / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
        }
        x[i] = y[0];
        v[i] = y[1];
        e[i] = y[2];
    }
}

/* ---------------------------------------------------------------------------------------------
 * Discrete adjoint of the integrator map for the per-particle window mean velocity
 *   J_i = (x_S - x_{S-W}) / (W dt).
 * The whole trajectory of a particle is stored (no checkpoints); lambda_k = dJ/dy_k is carried
 * from k = S down to 0 through the transposed Jacobian of the step, and the explicit parameter
 * derivatives of each step are accumulated. Gradient order:
 *   (U0, a, D, d2, q, c, gamma0, F0).
 *
 * With f the drift of Eqs. (1)-(2), J_f its Jacobian, f_th its parameter derivative and
 * g xi = (0, sigma xi, 0) the noise increment (sigma = sqrt(2 D dt)):
 *   EM    y' = y + f(y) dt + g xi
 *         lambda = lambda' + dt J_f(y)^T lambda'
 *         grad  += dt f_th(y)^T lambda' + lambda'_v xi dsigma/dtheta
 *   Heun  y~ = y + f(y) dt + g xi,   y' = y + (f(y) + f(y~)) dt/2 + g xi
 *         mu = J_f(y~)^T lambda',  nu = lambda' + dt mu
 *         lambda = lambda' + dt/2 (mu + J_f(y)^T nu)
 *         grad  += dt/2 f_th(y~)^T lambda' + dt/2 f_th(y)^T nu + (lambda'_v + dt/2 mu_v) xi dsigma/dth
 *
 * eps != 0 records the forward path under the rounding-sensitivity model (see perturb) and
 * linearises around that path, which measures how well-conditioned each particle's gradient is.
 * lookback = T > 0 (Euler-Maruyama only) computes the decayed estimator: J is written as
 * (1/W) sum of v_k for k >= wb (the same function of the EM path), each v_k's sensitivity
 * carried back with an extra factor rho = 1 - 1/T per step.
 * Returns -1 on bad input (D must be > 0 since dsigma/dD is singular at D = 0).
 * ------------------------------------------------------------------------------------------- */
enum { NGRAD = 8 };

/* J_f(y)^T w */
static void drift_jac_t(const orc_params *p, const double y[3], const double w[3], double out[3])
{
    const double x = y[0], v = y[1], e = y[2];
    out[0] = -d2U(p, x) * w[1];
    out[1] = w[0] + (p->d2 * e - p->gamma0) * w[1] - 2.0 * p->d2 * e * v * w[2];
    out[2] = p->d2 * v * w[1] - (p->c + p->d2 * v * v) * w[2];
}

/* g[j] += scale * f_theta_j(y)^T w for the drift-borne parameters (all but D) */
static void add_drift_param_grad(const orc_params *p, const double y[3], const double w[3],
                                 double scale, double g[NGRAD])
{
    const double x = y[0], v = y[1], e = y[2];
    const double th = 2.0 * ORC_PI * (x + p->phi);
    g[0] += scale * w[1] * (-2.0 * ORC_PI * (cos(th) + 2.0 * p->a * cos(2.0 * th)));
    g[1] += scale * w[1] * (-4.0 * ORC_PI * p->U0 * cos(2.0 * th));
    g[3] += scale * (w[1] * e * v - w[2] * e * v * v);
    g[4] += scale * w[2];
    g[5] += scale * w[2] * (-e);
    g[6] += scale * w[1] * (-v);
    g[7] += scale * w[1];
}

int orc_adjoint(const orc_params *p, int scheme, double dt, int64_t n_steps, int64_t window,
                uint64_t seed, uint32_t set, int64_t n, const uint32_t *ids, const double *x0,
                const double *v0, const double *e0, double *J, double *grad, double eps,
                int64_t lookback)
{
    if (!(dt > 0.0) || n_steps < 1 || window < 1 || window > n_steps || !(p->D > 0.0) ||
        (scheme != ORC_EM && scheme != ORC_HEUN) || lookback < 0 ||
        (lookback > 0 && scheme != ORC_EM))
        return -1;
    const double sig = sqrt(2.0 * p->D * dt);
    const double dsig_dD = sqrt(dt / (2.0 * p->D));
    const int64_t wb = n_steps - window;
    const double jscale = 1.0 / ((double)window * dt);
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t pid = ids ? ids[i] : (uint32_t)i;
        double *ty = malloc(sizeof(double) * 3 * (size_t)(n_steps + 1));
        double *tz = malloc(sizeof(double) * (size_t)n_steps);
        if (!ty || !tz) {
            free(ty); free(tz);
#pragma omp atomic write
            failed = 1;
            continue;
        }
        orc_normals(seed, pid, set, 0, n_steps, tz);
        double y[3] = {x0[i], v0[i], e0[i]};
        for (int64_t k = 0; k < n_steps; ++k) {
            memcpy(ty + 3 * k, y, sizeof y);
            one_step(p, scheme, dt, sig, tz[k], y);
            if (eps != 0.0)
                perturb(seed, pid, set, k, eps, y);
        }
        memcpy(ty + 3 * n_steps, y, sizeof y);
        J[i] = (ty[3 * n_steps] - ty[3 * wb]) * jscale;

        const int vform = lookback > 0;
        const double rho = vform ? 1.0 - 1.0 / (double)lookback : 1.0;
        double lam[3] = {vform ? 0.0 : jscale, 0.0, 0.0};
        double g[NGRAD] = {0};
        for (int64_t k = n_steps - 1; k >= 0; --k) {
            /* lam holds dJ/dy_{k+1}; the window-start position enters at index wb */
            if (k + 1 == wb && !vform)
                lam[0] -= jscale;
            const double *yk = ty + 3 * k;
            double nl[3], jt[3];
            if (scheme == ORC_EM) {
                add_drift_param_grad(p, yk, lam, dt, g);
                g[2] += lam[1] * tz[k] * dsig_dD;
                drift_jac_t(p, yk, lam, jt);
                for (int d = 0; d < 3; ++d)
                    nl[d] = lam[d] + dt * jt[d];
            } else {
                double f[3], yp[3];
                drift(p, yk[0], yk[1], yk[2], f);
                yp[0] = yk[0] + f[0] * dt;
                yp[1] = yk[1] + f[1] * dt + sig * tz[k];
                yp[2] = yk[2] + f[2] * dt;
                double mu[3], nu[3];
                drift_jac_t(p, yp, lam, mu);
                for (int d = 0; d < 3; ++d)
                    nu[d] = lam[d] + dt * mu[d];
                add_drift_param_grad(p, yp, lam, 0.5 * dt, g);
                add_drift_param_grad(p, yk, nu, 0.5 * dt, g);
                g[2] += (lam[1] + 0.5 * dt * mu[1]) * tz[k] * dsig_dD;
                drift_jac_t(p, yk, nu, jt);
                for (int d = 0; d < 3; ++d)
                    nl[d] = lam[d] + 0.5 * dt * (mu[d] + jt[d]);
            }
            if (vform) {
                lam[0] = rho * nl[0];
                lam[1] = rho * nl[1] + (k >= wb ? 1.0 / (double)window : 0.0);
                lam[2] = rho * nl[2];
            } else {
                memcpy(lam, nl, sizeof nl);
            }
        }
        for (int j = 0; j < NGRAD; ++j)
            grad[NGRAD * i + j] = g[j];
        free(ty); free(tz);
    }
    return failed ? -2 : 0;
}

/* ---------------------------------------------------------------------------------------------
 * Complex-step derivative (Squire & Trapp 1998): the same integrator run in complex arithmetic
 * with parameter `which` (0..7 = U0, a, D, d2, q, c, gamma0, F0) shifted by i*h. For an analytic
 * recursion Im(J(theta + i h))/h equals dJ/dtheta up to rounding, with no subtractive
 * cancellation. Forward mode and independent of the adjoint above; used to pin it.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    double complex U0, a, D, d2, q, c, gamma0, F0;
} cparams;

static void cdrift(const cparams *cp, double phi, double complex x, double complex v,
                   double complex e, double complex f[3])
{
    double complex th = 2.0 * ORC_PI * (x + phi);
    double complex dUx = 2.0 * ORC_PI * cp->U0 * (ccos(th) + 2.0 * cp->a * ccos(2.0 * th));
    f[0] = v;
    f[1] = cp->F0 - cp->gamma0 * v + cp->d2 * e * v - dUx;
    f[2] = cp->q - cp->c * e - cp->d2 * e * v * v;
}

int orc_complex_step(const orc_params *p, int scheme, int which, double h, double dt,
                     int64_t n_steps, int64_t window, uint64_t seed, uint32_t set, int64_t n,
                     const uint32_t *ids, const double *x0, const double *v0, const double *e0,
                     double *dJ, double *J_re)
{
    if (which < 0 || which >= NGRAD || !(dt > 0.0) || n_steps < 1 || window < 1 ||
        window > n_steps || (scheme != ORC_EM && scheme != ORC_HEUN))
        return -1;
    cparams cp = {p->U0, p->a, p->D, p->d2, p->q, p->c, p->gamma0, p->F0};
    double complex *field[NGRAD] = {&cp.U0, &cp.a, &cp.D, &cp.d2, &cp.q, &cp.c, &cp.gamma0, &cp.F0};
    *field[which] += I * h;
    const double complex sig = csqrt(2.0 * cp.D * dt);
    const int64_t wb = n_steps - window;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t pid = ids ? ids[i] : (uint32_t)i;
        double complex y[3] = {x0[i], v0[i], e0[i]}, xs = x0[i];
        double z[4];
        for (int64_t k = 0; k < n_steps; ++k) {
            if (k == wb)
                xs = y[0];
            if (k % 4 == 0)
                normals4(seed, pid, set, (uint32_t)(k / 4), z);
            double complex f[3], yp[3];
            cdrift(&cp, p->phi, y[0], y[1], y[2], f);
            yp[0] = y[0] + f[0] * dt;
            yp[1] = y[1] + f[1] * dt + sig * z[k % 4];
            yp[2] = y[2] + f[2] * dt;
            if (scheme == ORC_EM) {
                y[0] = yp[0]; y[1] = yp[1]; y[2] = yp[2];
            } else {
                double complex fp[3];
                cdrift(&cp, p->phi, yp[0], yp[1], yp[2], fp);
                y[0] = y[0] + 0.5 * (f[0] + fp[0]) * dt;
                y[1] = y[1] + 0.5 * (f[1] + fp[1]) * dt + sig * z[k % 4];
                y[2] = y[2] + 0.5 * (f[2] + fp[2]) * dt;
            }
        }
        if (wb == n_steps)
            xs = y[0];
        double complex Jc = (y[0] - xs) / ((double)window * dt);
        dJ[i] = cimag(Jc) / h;
        if (J_re)
            J_re[i] = creal(Jc);
    }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel regions (timing single-core against all-core). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
