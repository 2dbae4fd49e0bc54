// valu_rates.hip -- issue cost of the VALU instruction classes the integrator uses, on gfx950.
//
// Each kernel runs CHAINS independent dependency chains per lane of one instruction class for
// ITERS iterations, on a grid that fills every SIMD with 8 waves. The time per instruction,
// divided by the time per v_fma_f32 measured the same way, is that class's cost in full-rate
// VALU issue slots. Prints "name: ns_per_wave_instr_per_simd slots" lines.
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

template <int OP>
__global__ __launch_bounds__(256) void k_rate(float *out, float seedf, uint32_t seedu)
{
    float f[CHAINS];
    uint32_t u[CHAINS];
    for (int c = 0; c < CHAINS; ++c) {
        f[c] = seedf + 0.01f * (float)(threadIdx.x + c);
        u[c] = seedu + threadIdx.x * 7u + (uint32_t)c;
    }
    for (int it = 0; it < ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            if constexpr (OP == 0) {  // v_fma_f32
                f[c] = fmaf(f[c], 0.999f, 0.001f);
            } else if constexpr (OP == 1) {  // v_cos_f32
                f[c] = __builtin_amdgcn_cosf(f[c]);
            } else if constexpr (OP == 2) {  // v_sin_f32
                f[c] = __builtin_amdgcn_sinf(f[c]);
            } else if constexpr (OP == 3) {  // v_log_f32
                f[c] = __builtin_amdgcn_logf(f[c]);
            } else if constexpr (OP == 4) {  // v_sqrt_f32
                f[c] = __builtin_amdgcn_sqrtf(f[c]);
            } else if constexpr (OP == 5) {  // v_mad_u64_u32 (both halves kept)
                uint64_t r;
                asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(u[c]),
                             "v"(0xD2511F53u) : "vcc");
                u[c] = (uint32_t)r + (uint32_t)(r >> 32);
            } else if constexpr (OP == 6) {  // v_mul_hi_u32
                u[c] = __umulhi(u[c], 0xD2511F53u) + 1u;
            } else if constexpr (OP == 7) {  // v_bitop3_b32
                u[c] = __builtin_amdgcn_bitop3_b32(u[c], 0x9E3779B9u, (uint32_t)c, 0x96);
            } else if constexpr (OP == 8) {  // v_cvt_f32_u32
                f[c] = (float)(__float_as_uint(f[c]) >> 8);
            }
        }
    }
    float acc = 0.0f;
    for (int c = 0; c < CHAINS; ++c)
        acc += f[c] + (float)u[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// instructions per chain-iteration beyond the measured one (loop bookkeeping is SALU)
static const char *kNames[] = {"fma_f32", "cos_f32", "sin_f32", "log_f32", "sqrt_f32",
                               "mad_u64_u32+add", "mul_hi_u32+add", "bitop3_b32", "lshr+cvt_f32"};
static const double kInstr[] = {1, 1, 1, 1, 1, 2, 2, 1, 2};

template <int OP>
static double run(float *d_out, int grid, int block)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(k_rate<OP>, dim3(grid), dim3(block), 0, 0, d_out, 0.5f, 12345u);
    CHECK(hipEventRecord(a));
    const int reps = 5;
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_rate<OP>, dim3(grid), dim3(block), 0, 0, d_out, 0.5f, 12345u);
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipGetLastError());
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const int block = 256, grid = cus * 8;  // 8 waves per SIMD
    float *d_out = nullptr;
    CHECK(hipMalloc(&d_out, sizeof(float) * (size_t)grid * block));
    double ms[9];
    ms[0] = run<0>(d_out, grid, block);
    ms[1] = run<1>(d_out, grid, block);
    ms[2] = run<2>(d_out, grid, block);
    ms[3] = run<3>(d_out, grid, block);
    ms[4] = run<4>(d_out, grid, block);
    ms[5] = run<5>(d_out, grid, block);
    ms[6] = run<6>(d_out, grid, block);
    ms[7] = run<7>(d_out, grid, block);
    ms[8] = run<8>(d_out, grid, block);
    const double waves_per_simd = (double)grid * block / 64.0 / (cus * 4.0);
    const double instr_per_wave = (double)ITERS * CHAINS;
    std::printf("# device: %s, %d CUs, clock %d kHz\n", prop.gcnArchName, cus, prop.clockRate);
    std::printf("# grid %d x %d threads (%.0f waves/SIMD), %d chains x %d iterations per lane\n",
                grid, block, waves_per_simd, CHAINS, ITERS);
    const double ns_fma = ms[0] * 1e6 / (waves_per_simd * instr_per_wave * kInstr[0]);
    for (int i = 0; i < 9; ++i) {
        const double ns = ms[i] * 1e6 / (waves_per_simd * instr_per_wave * kInstr[i]);
        std::printf("%-16s %8.3f ms  %7.4f ns/wave-instr/SIMD  %5.2f slots (avg over %g instr)\n",
                    kNames[i], ms[i], ns, ns / ns_fma, kInstr[i]);
    }
    // cost of the class itself, with the companion full-rate op removed
    const double slot_ns = ns_fma;
    auto slots = [&](int i) { return ms[i] * 1e6 / (waves_per_simd * instr_per_wave) / slot_ns; };
    std::printf("fma_slot_ns: %.4f\n", slot_ns);
    std::printf("implied_clock_ghz: %.3f\n", 4.0 / slot_ns);
    const double trans = (slots(1) + slots(2) + slots(3) + slots(4)) / 4.0;
    std::printf("trans_slots: %.3f\n", trans);
    std::printf("mad64_slots: %.3f\n", slots(5) - 1.0);
    std::printf("mul_hi_slots: %.3f\n", slots(6) - 1.0);
    std::printf("bitop3_slots: %.3f\n", slots(7));
    CHECK(hipFree(d_out));
    return 0;
}
