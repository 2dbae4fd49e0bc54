// valu_rates.hip -- issue cost of the VALU instruction classes the integrator uses, on gfx950.
//
// Each kernel runs CHAINS independent dependency chains per lane of one instruction (or of a
// fixed pair of instructions) for ITERS iterations, on a grid of 256-thread blocks giving W waves
// per SIMD. The time per wave-instruction per SIMD, divided by that of v_fma_f32 at 8 waves per
// SIMD, is the cost of the class in FMA issue slots. Pairs show which classes overlap.
// Output: one line per measurement, then "key: value" summary lines.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CHAINS 8
#define ITERS 4096

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

enum Op {
    FMA, ADD, MUL, COS, LOG, SQRT, MAD64, MULHI, MULLO, BITOP3, ADDU, CVT, FMA64,
    MIX_FMA_COS, MIX_FMA_MAD64, MIX_FMA_BITOP3, MIX_COS_MAD64, FMAMK, N_OPS
};
static const char *kNames[N_OPS] = {
    "v_fma_f32(3v)", "v_add_f32", "v_mul_f32", "v_cos_f32", "v_log_f32", "v_sqrt_f32",
    "mad_u64+mov", "v_mul_hi_u32", "v_mul_lo_u32", "v_bitop3_b32", "v_add_u32",
    "v_cvt_f32_u32", "v_fma_f64", "fma+cos", "fma+mad64+mov", "fma+bitop3", "cos+mad64+mov", "v_fmamk_f32"};
// v_mad_u64_u32 chains carry one v_mov_b32 each (the zero high word of the addend)
static const int kInstr[N_OPS] = {1, 1, 1, 1, 1, 1, 2, 1, 1, 1, 1, 1, 1, 2, 3, 2, 3, 1};

__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c)
{
    return (uint64_t)a * (uint64_t)b + c;  // selects v_mad_u64_u32
}

template <int OP>
__global__ __launch_bounds__(256) void k_rate(float *out, float seedf, uint32_t seedu)
{
    float f[CHAINS];
    uint32_t u[CHAINS];
    uint64_t w[CHAINS];
    double d[CHAINS];
    const float g = seedf * 0.5f + (float)(threadIdx.x & 1), h = seedf * 0.25f;
    const uint32_t m = seedu | 1u;
    for (int c = 0; c < CHAINS; ++c) {
        f[c] = seedf + 0.01f * (float)(threadIdx.x + c);
        u[c] = seedu + threadIdx.x * 7u + (uint32_t)c;
        w[c] = u[c];
        d[c] = f[c];
    }
    for (int it = 0; it < ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            if constexpr (OP == FMA) f[c] = fmaf(f[c], g, h);
            else if constexpr (OP == ADD) f[c] = f[c] + g;
            else if constexpr (OP == MUL) f[c] = f[c] * g;
            else if constexpr (OP == COS) f[c] = __builtin_amdgcn_cosf(f[c]);
            else if constexpr (OP == LOG) f[c] = __builtin_amdgcn_logf(f[c]);
            else if constexpr (OP == SQRT) f[c] = __builtin_amdgcn_sqrtf(f[c]);
            else if constexpr (OP == MAD64) w[c] = mad64((uint32_t)w[c], m, w[c] >> 32);
            else if constexpr (OP == MULHI) u[c] = __umulhi(u[c], m);
            else if constexpr (OP == MULLO)  // asm: keeps the chain from being folded
                asm volatile("v_mul_lo_u32 %0, %1, %2" : "=v"(u[c]) : "v"(u[c]), "v"(m));
            else if constexpr (OP == BITOP3)
                u[c] = __builtin_amdgcn_bitop3_b32(u[c], m, (uint32_t)c, 0x96);
            else if constexpr (OP == ADDU)
                asm volatile("v_add_u32 %0, %1, %2" : "=v"(u[c]) : "v"(u[c]), "v"(m));
            else if constexpr (OP == CVT)
                asm volatile("v_cvt_f32_u32 %0, %1" : "=v"(f[c]) : "v"(f[c]));
            else if constexpr (OP == FMAMK) f[c] = fmaf(f[c], 0.999f, h);
            else if constexpr (OP == FMA64) d[c] = fma(d[c], (double)g, (double)h);
            if constexpr (OP == MIX_FMA_COS) {
                // independent FMA and cos chains, interleaved
                f[c] = fmaf(f[c], g, h);
                u[c] = __float_as_uint(__builtin_amdgcn_cosf(__uint_as_float(u[c])));
            } else if constexpr (OP == MIX_FMA_MAD64) {
                f[c] = fmaf(f[c], g, h);
                w[c] = mad64((uint32_t)w[c], m, w[c] >> 32);
            } else if constexpr (OP == MIX_FMA_BITOP3) {
                f[c] = fmaf(f[c], g, h);
                u[c] = __builtin_amdgcn_bitop3_b32(u[c], m, (uint32_t)c, 0x96);
            } else if constexpr (OP == MIX_COS_MAD64) {
                f[c] = __builtin_amdgcn_cosf(f[c]);
                w[c] = mad64((uint32_t)w[c], m, w[c] >> 32);
            }
        }
    }
    float acc = 0.0f;
    for (int c = 0; c < CHAINS; ++c)
        acc += f[c] + (float)u[c] + (float)(uint32_t)w[c] + (float)d[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

typedef void (*Kern)(float *, float, uint32_t);

static double time_kernel(Kern k, float *d_out, int grid)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, 0, d_out, 0.5f, 12345u);
    CHECK(hipEventRecord(a));
    const int reps = 5;
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, 0, d_out, 0.5f, 12345u);
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipGetLastError());
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

template <int... OPS>
struct Table {
    static constexpr Kern k[sizeof...(OPS)] = {k_rate<OPS>...};
};

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    float *d_out = nullptr;
    CHECK(hipMalloc(&d_out, sizeof(float) * (size_t)cus * 8 * 256));
    using T = Table<FMA, ADD, MUL, COS, LOG, SQRT, MAD64, MULHI, MULLO, BITOP3, ADDU, CVT, FMA64,
                    MIX_FMA_COS, MIX_FMA_MAD64, MIX_FMA_BITOP3, MIX_COS_MAD64, FMAMK>;
    std::printf("# device: %s, %d CUs, max clock %d kHz; %d chains x %d iterations per lane\n",
                prop.gcnArchName, cus, prop.clockRate, CHAINS, ITERS);
    const double instr_per_wave = (double)ITERS * CHAINS;
    double ns8[N_OPS];
    for (int wps : {1, 2, 4, 8}) {
        const int grid = cus * wps;  // 4 waves per block: wps waves per SIMD
        for (int op = 0; op < N_OPS; ++op) {
            if (wps != 8 && op != FMA && op != COS && op != MAD64 && op != FMAMK)
                continue;
            const double ms = time_kernel(T::k[op], d_out, grid);
            const double ns = ms * 1e6 / (wps * instr_per_wave * kInstr[op]);
            if (wps == 8)
                ns8[op] = ns;
            std::printf("%-14s waves/SIMD %d  %8.4f ms  %7.4f ns per wave-instr per SIMD\n",
                        kNames[op], wps, ms, ns);
        }
    }
    // reference slot: the fastest plain FP32 op (register-operand FMA is limited by VGPR reads)
    double fma = ns8[FMAMK];
    if (ns8[ADD] < fma) fma = ns8[ADD];
    if (ns8[MUL] < fma) fma = ns8[MUL];
    std::printf("fma_ns: %.4f\n", fma);
    std::printf("fma_cycles_at_max_clock: %.3f\n", fma * prop.clockRate * 1e-6);
    std::printf("trans_slots: %.3f\n", (ns8[COS] + ns8[LOG] + ns8[SQRT]) / 3.0 / fma);
    std::printf("mad64_slots: %.3f\n", (2.0 * ns8[MAD64] - ns8[ADDU]) / fma);
    std::printf("mul_hi_slots: %.3f\n", ns8[MULHI] / fma);
    std::printf("bitop3_slots: %.3f\n", ns8[BITOP3] / fma);
    std::printf("int_slots: %.3f\n", (ns8[ADDU] + ns8[CVT]) / 2.0 / fma);
    std::printf("fp32_addmul_slots: %.3f\n", (ns8[ADD] + ns8[MUL]) / 2.0 / fma);
    std::printf("pair_fma_cos_slots_per_instr: %.3f\n", ns8[MIX_FMA_COS] / fma);
    std::printf("pair_fma_mad64_slots_per_instr: %.3f\n", ns8[MIX_FMA_MAD64] / fma);
    CHECK(hipFree(d_out));
    return 0;
}
