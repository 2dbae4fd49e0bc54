// common.hpp -- host-side helpers shared by the entry points of libabp: argument validation,
// the gfx950 device check, conversion of the FP64 model parameters into the FP32 wavefront
// constants, and launch-shape selection.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/abp.h"
#include "device.hpp"

namespace abp {

constexpr int64_t kMaxStepIndex = int64_t(1) << 34;  // block counter n/4 fits one 32-bit word
constexpr int64_t kMaxParticles = int64_t(1) << 31;
constexpr int32_t kMaxBins = 4096;
constexpr double kPi = 3.14159265358979323846;

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

__host__ __device__ inline bool is_finite(double x) { return std::isfinite(x); }

__host__ __device__ inline bool params_ok(const abp_params &p)
{
    return is_finite(p.U0) && is_finite(p.a) && is_finite(p.phi) && is_finite(p.gamma0) && is_finite(p.F0) &&
           is_finite(p.d2) && is_finite(p.q) && is_finite(p.c) && is_finite(p.D) && p.D >= 0.0;
}

inline bool bins_ok(int32_t n_bins)
{
    return n_bins == 0 || (n_bins > 0 && n_bins <= kMaxBins && (n_bins & (n_bins - 1)) == 0);
}

// The library runs on gfx950 only; the answer is cached per device ordinal.
abp_status check_device();

// FP64 parameters -> FP32 wavefront constants. The phase enters only through cos/sin in
// revolutions (period 1), so it is reduced to [0, 1) in FP64 first: the kernels then add it to
// positions of magnitude <= 1/2 without losing low bits, and stay inside the hardware cosine's
// argument range for any finite phase. Phases already in [0, 1) are unchanged.
// The host (single-set calls) and the device (parameter tables in device memory) compute the
// same bits: every operation is a correctly rounded FP64 multiply or add taken in source order
// (contraction into fused multiply-adds is switched off), then one rounding to FP32.
__host__ __device__ inline Coef make_coef(const abp_params &p, double dt)
{
#pragma clang fp contract(off)
    Coef k;
    k.dt = (float)dt;
    k.half_dt = (float)(0.5 * dt);
    k.bm = (float)(-2.0 * 0.69314718055994530942 * (2.0 * p.D * dt));
    k.phi = (float)(p.phi - std::floor(p.phi));
    k.K1 = (float)(2.0 * kPi * p.U0);
    k.B = (float)(8.0 * kPi * p.U0 * p.a);
    k.FH = (float)(p.F0 + 4.0 * kPi * p.U0 * p.a);
    k.g0 = (float)p.gamma0;
    k.d2 = (float)p.d2;
    k.q = (float)p.q;
    k.c = (float)p.c;
    return k;
}

// The kernels compute with the FP32 coefficients: a parameter set and time step are accepted only
// if every coefficient is finite after the conversion and the FP32 time step is positive (finite
// FP64 values can overflow FP32, and a tiny dt can round to zero).
__host__ __device__ inline bool coef_ok(const Coef &k)
{
    const float f[] = {k.dt, k.half_dt, k.bm, k.phi, k.K1, k.B, k.FH, k.g0, k.d2, k.q, k.c};
    for (float x : f)
        if (!std::isfinite(x))
            return false;
    return k.dt > 0.0f;
}

inline Stream make_stream(uint64_t seed, uint32_t set)
{
    Stream s;
    s.k0 = (uint32_t)(seed & 0xFFFFFFFFull);
    s.k1 = (uint32_t)(seed >> 32);
    s.set = set;
    return s;
}

inline bool state_ok(const abp_state *s)
{
    if (!s || !s->d_cell || !s->d_xf || !s->d_v || !s->d_e || !s->d_lo)
        return false;
    if (!aligned(s->d_cell, 4) || !aligned(s->d_xf, 4) || !aligned(s->d_v, 4) ||
        !aligned(s->d_e, 4) || !aligned(s->d_lo, 4))
        return false;
    if (s->n < 1 || s->n > kMaxParticles)
        return false;
    return (uint64_t)s->id0 + (uint64_t)(s->n - 1) <= 0xFFFFFFFFull;
}

// Launch shape; loop = the advance() loop form: 1 or 2 blocks per trip, or kAhead.
struct Shape {
    int block, ppl, unroll, waves_per_simd, lookahead;
    int loop() const { return lookahead == 2 ? kAhead : unroll; }
};

inline bool resolve_tuning(const abp_tuning *t, Shape def, Shape &out)
{
    out = def;
    if (!t)
        return true;
    if (t->block)
        out.block = t->block;
    if (t->ppl)
        out.ppl = t->ppl;
    if (t->unroll)
        out.unroll = t->unroll;
    if (t->waves_per_simd)
        out.waves_per_simd = t->waves_per_simd;
    if (t->lookahead)
        out.lookahead = t->lookahead;
    if (out.block != 64 && out.block != 128 && out.block != 256)
        return false;
    if (out.ppl != 1 && out.ppl != 2)
        return false;
    if (out.unroll != 1 && out.unroll != 2)
        return false;
    if (out.lookahead < 0 || out.lookahead > 2 || (out.lookahead == 2 && out.unroll != 1))
        return false;
    return out.waves_per_simd >= 1 && out.waves_per_simd <= 8;
}

// Compute units of the current device (cached per device ordinal); 0 if the query fails.
int device_cus();

// The automatic look-ahead choice (lookahead = 0): on when `waves` wavefronts fill at most two per
// SIMD of the device, where a wavefront's own instruction stream is all a SIMD has to issue.
inline void resolve_lookahead(Shape &sh, int64_t waves)
{
    if (sh.lookahead != 0)
        return;
    const int cus = device_cus();
    sh.lookahead = (sh.unroll == 1 && cus > 0 && waves <= (int64_t)cus * 4 * 2) ? 2 : 1;
}

inline abp_status launch_status()
{
    return hipGetLastError() == hipSuccess ? ABP_OK : ABP_E_HIP;
}

constexpr int64_t n_tiles(int64_t n) { return (n + 63) / 64; }

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace abp
