// api.hip -- library-wide entry points: version and status strings, the device check, the
// initial condition and the raw Philox generator.
#include <atomic>

#include "common.hpp"
#include "reduce.hpp"

namespace abp {

abp_status check_device()
{
    static std::atomic<int> cache[64];  // 0 = unknown, 1 = gfx950, 2 = other (per device)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return ABP_E_DEVICE;
    if (dev >= 0 && dev < 64) {
        const int known = cache[dev].load(std::memory_order_relaxed);
        if (known)
            return known == 1 ? ABP_OK : ABP_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return ABP_E_DEVICE;
    const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev >= 0 && dev < 64)
        cache[dev].store(ok ? 1 : 2, std::memory_order_relaxed);
    return ok ? ABP_OK : ABP_E_DEVICE;
}

// x0 = (w0 >> 8) 2^-24 of Philox block (0, id, set, 1); v0 = e0 = 0.
int device_cus()
{
    static std::atomic<int> cache[64];  // 0 = unknown
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    if (dev >= 0 && dev < 64) {
        const int known = cache[dev].load(std::memory_order_relaxed);
        if (known)
            return known;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (dev >= 0 && dev < 64)
        cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

__global__ __launch_bounds__(256) void k_init_state(int32_t *cell, float *xf, float *v, float *e,
                                                    float *lo, int64_t n, uint32_t id0,
                                                    uint32_t set, uint32_t k0, uint32_t k1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const Philox4 r = philox4x32_10(0u, id0 + (uint32_t)i, set, kDomainInit, k0, k1);
    cell[i] = 0;
    xf[i] = (float)(r.w[0] >> 8) * 0x1p-24f;
    v[i] = 0.0f;
    e[i] = 0.0f;
    lo[i] = 0.0f;
    lo[n + i] = 0.0f;
    lo[2 * n + i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_philox(int64_t m, const uint32_t *ctr,
                                                const uint32_t *key, uint32_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m)
        return;
    const Philox4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                                    key[2 * i], key[2 * i + 1]);
    out[4 * i] = r.w[0];
    out[4 * i + 1] = r.w[1];
    out[4 * i + 2] = r.w[2];
    out[4 * i + 3] = r.w[3];
}

}  // namespace abp

using namespace abp;

extern "C" int abp_abi_version(void) { return ABP_ABI_VERSION; }

extern "C" const char *abp_status_str(int32_t status)
{
    // compared as an integer: a caller may pass any value, which an enum parameter of C++ could not
    // hold without undefined behaviour
    switch (status) {
    case ABP_OK: return "ok";
    case ABP_E_ARG: return "invalid argument";
    case ABP_E_HIP: return "HIP runtime error";
    case ABP_E_WORKSPACE: return "workspace too small";
    case ABP_E_DEVICE: return "device is not gfx950";
    }
    return "unknown status";
}

extern "C" abp_status abp_init_state(const abp_state *s, uint64_t seed, uint32_t set_id,
                                     void *stream)
{
    if (!state_ok(s))
        return ABP_E_ARG;
    if (abp_status st = check_device())
        return st;
    const Stream ks = make_stream(seed, set_id);
    const unsigned grid = (unsigned)((s->n + 255) / 256);
    hipLaunchKernelGGL(k_init_state, dim3(grid), dim3(256), 0, as_stream(stream), s->d_cell,
                       s->d_xf, s->d_v, s->d_e, s->d_lo, s->n, s->id0, set_id, ks.k0, ks.k1);
    return launch_status();
}

extern "C" abp_status abp_philox(int64_t m, const uint32_t *d_ctr, const uint32_t *d_key,
                                 uint32_t *d_out, void *stream)
{
    if (m < 1 || m > (int64_t(1) << 32) || !d_ctr || !d_key || !d_out || !aligned(d_ctr, 4) ||
        !aligned(d_key, 4) || !aligned(d_out, 4))
        return ABP_E_ARG;
    if (abp_status st = check_device())
        return st;
    const unsigned grid = (unsigned)((m + 255) / 256);
    hipLaunchKernelGGL(k_philox, dim3(grid), dim3(256), 0, as_stream(stream), m, d_ctr, d_key,
                       d_out);
    return launch_status();
}
