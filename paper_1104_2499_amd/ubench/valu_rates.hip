// valu_rates.hip -- issue cost of the VALU instruction classes the integrator uses, on gfx950.
//
// Each kernel runs CHAINS independent dependency chains per lane of one instruction (or of a
// fixed pair of instructions) for ITERS iterations, on a grid of 256-thread blocks giving W waves
// per SIMD. The time per wave-instruction per SIMD, divided by that of v_fma_f32 at 8 waves per
// SIMD, is the cost of the class in FMA issue slots. Pairs show which classes overlap.
// Output: one line per measurement, then "key: value" summary lines (the mix lines last).
// With --mix, only the mix lines.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

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

// ---------------------------------------------------------------------------------------------
// The integrators' own instruction mix, replayed without dependencies: the measured ceiling of
// that mix. Each string is the instruction sequence of one loop trip of k_integrate -- one aligned
// 8-step span, two noise blocks, one particle per lane, in-place noise loop -- in program order as
// hipcc -O3 compiles it for gfx950, one letter per instruction:
//   F v_fma/v_fmac_f32 with an SGPR operand    G v_fma/v_fmac_f32 on three VGPRs
//   A v_add/v_sub_f32     M v_mul_f32 with an SGPR    N v_mul_f32 on two VGPRs
//   C v_cos_f32   S v_sin_f32   L v_log_f32   Q v_sqrt_f32
//   D v_mad_u64_u32   X v_bitop3_b32   x v_xor_b32   B v_alignbit_b32   V v_mov (32 or 64 bit)
//   R v_rndne_f32   I v_cvt_i32_f32   U v_add_u32 / v_add_co_u32   K v_cmp_ge_i64
//   s a scalar ALU instruction
// (tests/test_isa_constraints.py checks that the class counts still match the library's loops).
// k_mix issues the same sequence on register chains that never wait for each other (each class
// rotates over a few registers), so its time per trip is the issue cost of the mix alone.
// ---------------------------------------------------------------------------------------------
static constexpr char kHeunTrip[] =
    "sssssssVVAsssxAAssssDCMsxAFFssxDsCsFsDsxsXxDsFDDXxFFXXDDFGDDXXFXXDDDDXXXXDDDDXXX"
    "XDDDDXXXXDDDDXXXXDDDBXXXBADBBXAABLLALLBMMCSCBQQMCSQBMCSSQNNNFNNFFANNNGMAFFAFFAAA"
    "CFAFCAMFFFFFGFFFFAFGMAFFAFFAAACFAFCAMFFFFFGFFFFAFGMAFFAFFAAACFAFCAMFFFFFGFFFFAFG"
    "MAFFAFFAAACFAFCAMFFFFFGFFFFAFGMAFFAFFAAACFAFCAMFFFFFGFFFFAFGMAFFAFFAAACFAFCAMFFF"
    "FFGFFFFAFGMAFFAFFAAACFAFCAMFFFFFGFFFFAFGAMFAFFAFARAAAIAFAAUAAssAAUs";
static constexpr char kEmTrip[] =
    "sssssVssxVsAAsDsAsMsAsCxFxFFsssDFDAssssCsxXxsFDsFDDXxFXXDDGDDFXXXXFDDDDXXXXDDDDX"
    "XXXDDDDXXXXDDDDXXXXDDDBXXXBADBBXAALLBABLMMCSCQQBMSLCSQNNNFAAFABMNNNGMFCSQFFAFACF"
    "AMFNNAFAFFFCFGFFAAFFAFGMFFFAFACFAMFAFAFFFCFGFFAAFFAFGMFFFAFACFAFAAMFCFFFFGFFAAFF"
    "AFGMFFFAFARAAIAFAAUAAssAAUs";

constexpr char trip_op(int kind, int i) { return kind == 0 ? kHeunTrip[i] : kEmTrip[i]; }
constexpr int trip_len(int kind) { return kind == 0 ? (int)sizeof(kHeunTrip) - 1 : (int)sizeof(kEmTrip) - 1; }

// Occurrences of the letter of instruction i among instructions 0..i-1: each class rotates over
// its own registers by this ordinal, so that consecutive instructions of a class never touch the
// same register.
constexpr int trip_ordinal(int kind, int i)
{
    int n = 0;
    for (int j = 0; j < i; ++j)
        n += trip_op(kind, j) == trip_op(kind, i);
    return n;
}

constexpr bool is_trans(char c) { return c == 'C' || c == 'S' || c == 'L' || c == 'Q'; }

// Transcendentals (of any of the four letters) among instructions 0..i-1.
constexpr int trans_ordinal(int kind, int i)
{
    int n = 0;
    for (int j = 0; j < i; ++j)
        n += is_trans(trip_op(kind, j));
    return n;
}

// Register chains (4 for the frequent classes, 2 for the rare ones) and loop-invariant operands.
// Every instruction reads only invariants, scalars and its own chain, which it last wrote several
// instructions of its class earlier: no instruction waits for another, and the compiler has no
// reason to pad the asm with wait states. VGPRs stay under 64, so eight wavefronts fit a SIMD.
struct MixRegs {
    float fF[4], fA[4], fT[4], fG[2], fM[2], fN[2], fR[2];
    uint32_t uX[4], uI[2], uD[2];
    uint64_t wD[4];
    float cV[4];     // invariant FP32 operands
    uint32_t cU[4];  // invariant integer operands
    uint64_t cW;     // invariant 64-bit operand
    uint32_t sc[4];
    float g;
    uint32_t k;
    int64_t lim;
};

// Instruction I of the trip, then the rest (unrolled at compile time).
template <int KIND, int I>
__device__ __forceinline__ void emit(MixRegs &r)
{
    if constexpr (I < trip_len(KIND)) {
        constexpr char op = trip_op(KIND, I);
        constexpr int o = trip_ordinal(KIND, I), c4 = o & 3, c2 = o & 1, v = I & 3;
        if constexpr (op == 'F')
            asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(r.fF[c4]) : "v"(r.cV[v]), "s"(r.g));
        else if constexpr (op == 'G')
            asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(r.fG[c2]) : "v"(r.cV[v]), "v"(r.cV[(v + 1) & 3]));
        else if constexpr (op == 'A')
            asm volatile("v_add_f32 %0, %1, %0" : "+v"(r.fA[c4]) : "v"(r.cV[v]));
        else if constexpr (op == 'M')
            asm volatile("v_mul_f32 %0, %1, %0" : "+v"(r.fM[c2]) : "s"(r.g));
        else if constexpr (op == 'N')
            asm volatile("v_mul_f32 %0, %1, %0" : "+v"(r.fN[c2]) : "v"(r.cV[v]));
        else if constexpr (op == 'C' || op == 'S' || op == 'L' || op == 'Q') {
            constexpr int t = trans_ordinal(KIND, I) & 3;  // one rotation over all four letters
            if constexpr (op == 'C')
                asm volatile("v_cos_f32 %0, %0" : "+v"(r.fT[t]));
            else if constexpr (op == 'S')
                asm volatile("v_sin_f32 %0, %0" : "+v"(r.fT[t]));
            else if constexpr (op == 'L')
                asm volatile("v_log_f32 %0, %0" : "+v"(r.fT[t]));
            else
                asm volatile("v_sqrt_f32 %0, %0" : "+v"(r.fT[t]));
        } else if constexpr (op == 'D')  // the carry goes to a reserved SGPR pair nothing reads
            asm volatile("v_mad_u64_u32 %0, s[60:61], %1, %2, 0"
                         : "=v"(r.wD[c4]) : "v"(r.cU[v]), "s"(r.k) : "s60", "s61");
        else if constexpr (op == 'X')
            asm volatile("v_bitop3_b32 %0, %1, %0, %2 bitop3:0x96" : "+v"(r.uX[c4]) : "v"(r.cU[v]), "s"(r.k));
        else if constexpr (op == 'x')
            asm volatile("v_xor_b32 %0, %1, %0" : "+v"(r.uI[c2]) : "s"(r.k));
        else if constexpr (op == 'B')
            asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(r.uI[c2]) : "s"(r.k));
        else if constexpr (op == 'V')
            asm volatile("v_mov_b32 %0, %1" : "=v"(r.uD[c2]) : "v"(r.cU[v]));
        else if constexpr (op == 'R')
            asm volatile("v_rndne_f32 %0, %0" : "+v"(r.fR[c2]));
        else if constexpr (op == 'I')
            asm volatile("v_cvt_i32_f32 %0, %1" : "=v"(r.uD[c2]) : "v"(r.cV[v]));
        else if constexpr (op == 'U')
            asm volatile("v_add_u32 %0, %1, %0" : "+v"(r.uI[c2]) : "v"(r.cU[v]));
        else if constexpr (op == 'K')
            asm volatile("v_cmp_ge_i64 vcc, %0, %1" : : "s"(r.lim), "v"(r.cW) : "vcc");
        else if constexpr (op == 's')  // one scalar ALU op (s_mul_i32) in plain code: SALU writes in
            r.sc[c4] *= r.sc[c4];         // asm make the compiler pad later statements with nops
        emit<KIND, I + 1>(r);
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_mix(float *out, float seedf, uint32_t seedu, int iters)
{
    MixRegs r;
    for (int c = 0; c < 4; ++c)
        r.sc[c] = seedu + (uint32_t)c;
    r.g = seedf * 0.5f;
    r.k = seedu | 1u;
    r.lim = (int64_t)seedu << 20;
    r.cW = (uint64_t)threadIdx.x << 7;
    for (int c = 0; c < 4; ++c) {
        r.cV[c] = seedf + 0.001f * (float)(threadIdx.x + 3 * c);
        r.cU[c] = seedu ^ (threadIdx.x * 0x9E3779B9u + (uint32_t)c);
        r.fF[c] = seedf + 0.01f * (float)(threadIdx.x + c);
        r.fA[c] = r.fF[c] + 1.0f;
        r.fT[c] = r.fF[c] * 0.5f;
        r.uX[c] = seedu + threadIdx.x * 7u + (uint32_t)c;
        r.wD[c] = r.uX[c];
    }
    for (int c = 0; c < 2; ++c) {
        r.fG[c] = r.fF[c] + 2.0f;
        r.fM[c] = r.fF[c] + 3.0f;
        r.fN[c] = r.fF[c] + 4.0f;
        r.fR[c] = r.fF[c] + 5.0f;
        r.uI[c] = r.uX[c] ^ 0x5555u;
        r.uD[c] = r.uX[c] + 11u;
    }
    for (int it = 0; it < iters; ++it)
        emit<KIND, 0>(r);
    float acc = 0.0f;
    for (int c = 0; c < 4; ++c)
        acc += (float)r.sc[c] + r.fF[c] + r.fA[c] + r.fT[c] + (float)r.uX[c] + (float)(uint32_t)r.wD[c];
    for (int c = 0; c < 2; ++c)
        acc += r.fG[c] + r.fM[c] + r.fN[c] + r.fR[c] + (float)(r.uD[c] ^ r.uI[c]);
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

static double time_mix(int kind, float *d_out, int grid, int iters)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    auto launch = [&]() {
        if (kind == 0)
            hipLaunchKernelGGL(k_mix<0>, dim3(grid), dim3(256), 0, 0, d_out, 0.5f, 12345u, iters);
        else
            hipLaunchKernelGGL(k_mix<1>, dim3(grid), dim3(256), 0, 0, d_out, 0.5f, 12345u, iters);
    };
    launch();
    CHECK(hipEventRecord(a));
    const int reps = 5;
    for (int r = 0; r < reps; ++r)
        launch();
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipGetLastError());
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
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

// Per-class issue costs: one line per measurement, then the summary lines.
static void class_rates(const hipDeviceProp_t &prop, float *d_out)
{
    using T = Table<FMA, ADD, MUL, COS, LOG, SQRT, MAD64, MULHI, MULLO, BITOP3, ADDU, CVT, FMA64,
                    MIX_FMA_COS, MIX_FMA_MAD64, MIX_FMA_BITOP3, MIX_COS_MAD64, FMAMK>;
    const int cus = prop.multiProcessorCount;
    const double instr_per_wave = (double)ITERS * CHAINS;
    double ns8[N_OPS] = {};
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
}

int main(int argc, char **argv)
{
    const bool mix_only = argc > 1 && std::strcmp(argv[1], "--mix") == 0;
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    float *d_out = nullptr;
    CHECK(hipMalloc(&d_out, sizeof(float) * (size_t)cus * 8 * 256));
    std::printf("# device: %s, %d CUs, max clock %d kHz; %d chains x %d iterations per lane\n",
                prop.gcnArchName, cus, prop.clockRate, CHAINS, ITERS);
    if (!mix_only)
        class_rates(prop, d_out);
    // the integrators' instruction mix: time per 8-step trip per wave per SIMD, by residency
    const int mix_iters = 1024;
    for (int kind = 0; kind < 2; ++kind) {
        const char *name = kind == 0 ? "heun" : "em";
        for (int wps : {1, 2, 4, 8}) {
            const double ms = time_mix(kind, d_out, cus * wps, mix_iters);
            const double ns = ms * 1e6 / ((double)wps * mix_iters);
            std::printf("mix_%s_trip_ns_w%d: %.4f\n", name, wps, ns);
        }
    }
    CHECK(hipFree(d_out));
    return 0;
}
