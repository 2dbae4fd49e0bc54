// device.hpp -- per-lane building blocks of the ABP integrator on gfx950.
//
// One particle (or two, PPL = 2) per lane; the state (cell, xf, v, e) lives in VGPRs for the whole
// launch. Everything uniform across a wavefront (model constants, Philox key schedule, step
// indices) is computed from kernel arguments and stays in SGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abp {

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each multiplies words 0 and 2 by
// the round constants, returning the high halves xor-ed with the neighbouring word and the key,
// and the low halves as the new words 1 and 3; the key is bumped by the Weyl increments between
// rounds. Words whose inputs are wavefront-uniform (the step block, set id and domain) stay on
// the scalar unit for the first rounds; the rest is v_mad_u64_u32 + v_bitop3_b32 per word pair.
// ---------------------------------------------------------------------------------------------
struct Philox4 {
    uint32_t w[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0, n2;
        if (r < 3) {
            // counter words still partly wavefront-uniform: let the scalar unit take its share
            n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        } else {
            // three-input xor in one VALU op (gfx950 v_bitop3_b32, truth table 0x96)
            n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
        }
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

enum : uint32_t { kDomainNoise = 0u, kDomainInit = 1u };

// ---------------------------------------------------------------------------------------------
// Box-Muller on 23-bit uniforms, with the noise amplitude folded in: returns sigma*z0, sigma*z1.
// One v_alignbit_b32 turns a Philox word w into y = 1 + (w >> 9) 2^-23 in [1, 2) (the word's top
// 23 bits under the exponent of 1.0). Then u1 = 2 - y1 in (0, 1] exactly, and because v_sin_f32 /
// v_cos_f32 take their argument in revolutions (period 1), sin(2 pi u2) = v_sin_f32(y2) with
// u2 = y2 - 1 in [0, 1). v_log_f32 is log2, so sigma rho = sqrt(bm * log2 u1) with the
// wavefront-uniform bm = -2 ln2 sigma^2.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float unit_interval_1_2(uint32_t w)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u));
}

__device__ __forceinline__ void box_muller_scaled(uint32_t wa, uint32_t wb, float bm, float &za,
                                                  float &zb)
{
    const float u1 = 2.0f - unit_interval_1_2(wa);
    const float y2 = unit_interval_1_2(wb);
    const float s = __builtin_amdgcn_sqrtf(bm * __builtin_amdgcn_logf(u1));
    za = s * __builtin_amdgcn_cosf(y2);
    zb = s * __builtin_amdgcn_sinf(y2);
}

// Noise block b of particle `pid`: sigma * (z0, z1, z2, z3) for steps 4b .. 4b+3.
struct Noise4 {
    float z[4];
};

__device__ __forceinline__ Noise4 noise_block(uint32_t blk, uint32_t pid, uint32_t set,
                                              uint32_t k0, uint32_t k1, float bm)
{
    const Philox4 r = philox4x32_10(blk, pid, set, kDomainNoise, k0, k1);
    Noise4 n;
    box_muller_scaled(r.w[0], r.w[1], bm, n.z[0], n.z[1]);
    box_muller_scaled(r.w[2], r.w[3], bm, n.z[2], n.z[3]);
    return n;
}

// ---------------------------------------------------------------------------------------------
// Drift of Eqs. (1)-(3) in FP32, wavefront-uniform coefficients, at the phase-shifted position
// xs = x + phi (in revolutions: only its fractional part matters).
//   U'(x) = 2 pi U0 [cos th + 2a cos 2th], th = 2 pi xs; with c = cos th and the double angle
//   cos 2th = 2c^2 - 1:  F0 - U'(x) = (F0 + 4 pi U0 a) - c (2 pi U0 + 8 pi U0 a c).
//   f_v = F0 - U'(x) + (d2 e - gamma0) v,   f_e = q - e (c + d2 v^2).
// ---------------------------------------------------------------------------------------------
struct Coef {
    float dt, half_dt, bm, phi;  // bm = -2 ln2 sigma^2, sigma = sqrt(2 D dt)
    float K1;   // 2 pi U0
    float B;    // 8 pi U0 a
    float FH;   // F0 + 4 pi U0 a
    float g0, d2, q, c;
};

// The drift from c = cos th (the adjoint's reverse sweep re-evaluates it from a staged cosine and
// gets the forward's bits).
__device__ __forceinline__ void drift_cos(const Coef &k, float cth, float v, float e, float &fv,
                                          float &fe)
{
    const float fu = fmaf(-cth, fmaf(k.B, cth, k.K1), k.FH);
    fv = fmaf(fmaf(k.d2, e, -k.g0), v, fu);
    fe = fmaf(-e, fmaf(k.d2 * v, v, k.c), k.q);
}

__device__ __forceinline__ void drift(const Coef &k, float xs, float v, float e, float &fv,
                                      float &fe)
{
    drift_cos(k, __builtin_amdgcn_cosf(xs), v, e, fv, fe);
}

// The stochastic Heun predictor's velocity and energy from the drift (fv0, fe0) at the current
// point: the expressions step_heun uses (the adjoint recomputes them with the same bits).
__device__ __forceinline__ void heun_predictor_ve(const Coef &k, float vc, float ec, float fv0,
                                                  float fe0, float zs, float &vp, float &ep)
{
    vp = vc + fmaf(fv0, k.dt, zs);
    ep = fmaf(fe0, k.dt, ec);
}

// ---------------------------------------------------------------------------------------------
// Particle state as a float-float pair per coordinate (the single-precision remedy for adding
// small increments to large values): x = cell + xf + lx, v = v + lv, e = e + le.
// Within an aligned span of kSpan = 8 steps (two noise blocks) the high parts (cell, xf, v, e) stay
// fixed and every increment goes into the low part, which starts the span holding the previous
// rounding error; after the span's last step each pair is renormalised by Fast2Sum (exact
// whenever the high part is the larger) and the nearest integer of xf moves into the cell,
// exactly. The drift sees the rounded sums (high + low). A state stored mid-span is resumed bit
// for bit.
// ---------------------------------------------------------------------------------------------
struct Particle {
    int32_t cell;
    float xf, v, e;
    float lx, lv, le;
};

// Euler-Maruyama: every drift at the old state; zs = sigma * xi_n; xb = xf + phi of the block.
__device__ __forceinline__ void step_em(const Coef &k, Particle &p, float xb, float zs)
{
    const float xc = xb + p.lx, vc = p.v + p.lv, ec = p.e + p.le;
    float fv, fe;
    drift(k, xc, vc, ec, fv, fe);
    p.lx = fmaf(vc, k.dt, p.lx);
    p.lv = p.lv + fmaf(fv, k.dt, zs);
    p.le = fmaf(fe, k.dt, p.le);
}

// Stochastic Heun for additive noise: Euler predictor with the same normal, then the
// trapezoidal average of the two drifts.
__device__ __forceinline__ void step_heun(const Coef &k, Particle &p, float xb, float zs)
{
    const float xc = xb + p.lx, vc = p.v + p.lv, ec = p.e + p.le;
    float fv0, fe0, fv1, fe1;
    drift(k, xc, vc, ec, fv0, fe0);
    const float xp = fmaf(vc, k.dt, xc);
    float vp, ep;
    heun_predictor_ve(k, vc, ec, fv0, fe0, zs, vp, ep);
    drift(k, xp, vp, ep, fv1, fe1);
    p.lx = fmaf(vc + vp, k.half_dt, p.lx);
    p.lv = p.lv + fmaf(fv0 + fv1, k.half_dt, zs);
    p.le = fmaf(fe0 + fe1, k.half_dt, p.le);
}

template <int SCHEME>
__device__ __forceinline__ void step(const Coef &k, Particle &p, float xb, float zs)
{
    if constexpr (SCHEME == 0)
        step_em(k, p, xb, zs);
    else
        step_heun(k, p, xb, zs);
}

__device__ __forceinline__ void renorm(float &hi, float &lo)
{
    const float t = hi + lo;
    lo = lo - (t - hi);
    hi = t;
}

// Steps between renormalisations: two noise blocks. (The low parts then hold at most eight
// increments; the span end's fixed cost -- three Fast2Sums, the wrap, the phase -- is paid once per
// eight steps.)
constexpr int kSpan = 8;

// End of an aligned span (after absolute step 8b+7): renormalise the pairs, then move the nearest
// integer of xf into the cell, leaving xf in [-1/2, 1/2]. For a binary float |x| < 2^23 the
// difference x - rint(x) is exactly representable (it keeps bits of x below the units place), so
// the wrap loses nothing and needs no error term. x leaves [-1/2, 1/2] by at most a few |v| dt per
// span, and cos (in revolutions) is periodic.
__device__ __forceinline__ void end_span(Particle &p)
{
    renorm(p.xf, p.lx);
    renorm(p.v, p.lv);
    renorm(p.e, p.le);
    const float r = __builtin_rintf(p.xf);
    p.xf -= r;
    p.cell += (int32_t)r;
}

__device__ __forceinline__ float pick(const Noise4 &n, uint32_t j)
{
    return j == 0 ? n.z[0] : j == 1 ? n.z[1] : j == 2 ? n.z[2] : n.z[3];
}

// Wavefront-uniform description of one particle set's noise and steps.
struct Stream {
    uint32_t k0, k1;  // Philox key
    uint32_t set;
};

// One aligned span of eight steps of one particle with the noise of its two blocks, then the span
// end.
template <int SCHEME>
__device__ __forceinline__ void span_steps(const Coef &k, Particle &p, const Noise4 &z0,
                                           const Noise4 &z1)
{
    const float xb = p.xf + k.phi;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        step<SCHEME>(k, p, xb, z0.z[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        step<SCHEME>(k, p, xb, z1.z[j]);
    end_span(p);
}

// Steps n .. lim-1 of one particle, one at a time, all inside one span (lim <= the span's end):
// each noise block is drawn as it is entered, and the span ends if lim closes it.
template <int SCHEME>
__device__ __forceinline__ void partial_steps(const Coef &k, const Stream &s, uint32_t pid,
                                              Particle &p, int64_t n, int64_t lim)
{
    const float xb = p.xf + k.phi;
    Noise4 z = noise_block((uint32_t)(n >> 2), pid, s.set, s.k0, s.k1, k.bm);
    for (int64_t m = n; m < lim; ++m) {
        if ((m & 3) == 0 && m != n)
            z = noise_block((uint32_t)(m >> 2), pid, s.set, s.k0, s.k1, k.bm);
        step<SCHEME>(k, p, xb, pick(z, (uint32_t)(m & 3)));
    }
    if ((lim & (kSpan - 1)) == 0)
        end_span(p);
}

// Advance PPL particles of one lane from absolute step n to `stop` (both wavefront-uniform).
// Spans of eight steps aligned on absolute indices take the fast path; a call that starts or ends
// inside a span handles its partial span step by step. Span ends (renormalisation and wrap)
// happen only after absolute steps 8b+7, so any split of a run into calls gives bit-identical
// states.
// Loop forms (all compute the same values): LOOP = 1, each span's noise right before its steps;
// LOOP = 2, two spans' noise per loop trip, then their steps; LOOP = kAhead, the noise of span
// b+1 (Philox and Box-Muller, which do not depend on the state) computed while span b steps, so
// that the two dependency chains overlap in one instruction stream -- for launches that hold one
// or two wavefronts per SIMD, where a wavefront's own instruction stream is all the SIMD has.
// Loop counters are 32-bit (spans of one call < 2^31), so that loop control stays scalar.
constexpr int kAhead = 3;

template <int SCHEME, int PPL, int UNROLL>
__device__ __forceinline__ void advance(const Coef &k, const Stream &s, const uint32_t (&pid)[PPL],
                                        Particle (&p)[PPL], int64_t &n, int64_t stop)
{
    // leading partial span
    if (n < stop && (n & (kSpan - 1))) {
        const int64_t end = (n | (kSpan - 1)) + 1;
        const int64_t lim = stop < end ? stop : end;
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            partial_steps<SCHEME>(k, s, pid[q], p[q], n, lim);
        n = lim;
    }
    // aligned spans
    const uint32_t nsp = (uint32_t)((stop - n) >> 3);
    uint32_t blk = (uint32_t)(n >> 2);
    if constexpr (UNROLL == kAhead) {
        if (nsp > 0) {
            Noise4 z0[PPL], z1[PPL];
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                z0[q] = noise_block(blk, pid[q], s.set, s.k0, s.k1, k.bm);
                z1[q] = noise_block(blk + 1, pid[q], s.set, s.k0, s.k1, k.bm);
            }
            for (uint32_t b = 1; b < nsp; ++b) {
                Noise4 n0[PPL], n1[PPL];
#pragma unroll
                for (int q = 0; q < PPL; ++q) {
                    n0[q] = noise_block(blk + 2, pid[q], s.set, s.k0, s.k1, k.bm);
                    n1[q] = noise_block(blk + 3, pid[q], s.set, s.k0, s.k1, k.bm);
                }
#pragma unroll
                for (int q = 0; q < PPL; ++q) {
                    span_steps<SCHEME>(k, p[q], z0[q], z1[q]);
                    z0[q] = n0[q];
                    z1[q] = n1[q];
                }
                blk += 2;
            }
            // the last aligned span (a trailing partial span draws its own noise)
#pragma unroll
            for (int q = 0; q < PPL; ++q)
                span_steps<SCHEME>(k, p[q], z0[q], z1[q]);
            blk += 2;
        }
    } else {
        uint32_t b = 0;
        for (; b + UNROLL <= nsp; b += UNROLL) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
                for (int q = 0; q < PPL; ++q) {
                    const Noise4 z0 = noise_block(blk + 2 * u, pid[q], s.set, s.k0, s.k1, k.bm);
                    const Noise4 z1 =
                        noise_block(blk + 2 * u + 1, pid[q], s.set, s.k0, s.k1, k.bm);
                    span_steps<SCHEME>(k, p[q], z0, z1);
                }
            }
            blk += 2 * UNROLL;
        }
        for (; b < nsp; ++b) {
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                const Noise4 z0 = noise_block(blk, pid[q], s.set, s.k0, s.k1, k.bm);
                const Noise4 z1 = noise_block(blk + 1, pid[q], s.set, s.k0, s.k1, k.bm);
                span_steps<SCHEME>(k, p[q], z0, z1);
            }
            blk += 2;
        }
    }
    n += (int64_t)nsp << 3;
    // trailing partial span (its end is taken by the call that finishes the span)
    if (n < stop) {
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            partial_steps<SCHEME>(k, s, pid[q], p[q], n, stop);
        n = stop;
    }
}

// ---------------------------------------------------------------------------------------------
// Reduction helpers
// ---------------------------------------------------------------------------------------------
// Butterfly sum over the 64 lanes of a wavefront in a fixed order (every lane ends with the total).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        x += __shfl_xor(x, m, 64);
    return x;
}

// Position cell + xf + lx in FP64 (evaluated left to right).
__device__ __forceinline__ double position64(int32_t cell, float xf, float lx)
{
    return ((double)cell + (double)xf) + (double)lx;
}

// Histogram bin of a position, decided in FP64: floor(n_bins * (x - floor x)), clamped.
__device__ __forceinline__ int32_t hist_bin(double x, int32_t n_bins)
{
    const double frac = x - floor(x);
    if (!(frac >= 0.0))
        return 0;  // not reached for finite positions
    const int32_t b = (int32_t)floor(frac * (double)n_bins);
    return b >= n_bins ? n_bins - 1 : b;
}

}  // namespace abp
