// op_rates.hip - per-instruction issue costs on gfx950, measured.
//
// Measurement code, not part of the integrator: it gives the denominators of
// the issue-rate rooflines (how many SIMD cycles one wave64 instruction of
// each class occupies) and checks the rate assumptions of the cost model
// (transcendentals and 32-bit multiplies at a quarter or half of the FMA
// rate, whether a DPP operand costs extra, whether transcendental and
// full-rate instructions overlap).
//
// Each kernel runs `iters` iterations of a block of one instruction class
// (or one fixed mix) over 8 independent register chains, written as
// one-instruction inline assembly, so the compiler neither drops nor
// rewrites any of them.  Chains are independent of each other, so
// consecutive instructions never wait on each other's results; DPP forms
// read a register the loop never writes.  One workgroup runs per CU with W
// waves on each of its four SIMDs; after a barrier every wave reads the
// shader clock (clock64) before and after its loop, and the host takes a
// workgroup's span (latest end - earliest start) as the SIMD cycles its
// W waves' instructions took: cycles per wave-instruction = span / (W x
// instructions per wave).  W = 1 shows what one wave alone can issue, W = 4
// what the SIMD can.  The binary64 library functions (sin, cos, log, sqrt
// of the device math library) are timed the same way over dependent call
// chains, per call, and so are the coupled kernels' own binary64 sine of a
// phase difference and their Box-Muller pair beside the library-function
// one.
//
// Only ALU work, one store per lane (to a buffer of one float per lane) and
// two per wave (its two clock readings).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "noise.hpp"
#include "phase64.hpp"

namespace {

constexpr int kChains = 8;
constexpr int kRepeat = 4;  // blocks of 8 per loop iteration

enum Op : int {
    kFmaF32 = 0,
    kAddF32,
    kMulF32,
    kSubDppF32,     // v_sub_f32 with a DPP row rotation on its first operand
    kMovDpp,        // v_mov_b32 with a DPP row rotation
    kSinF32,
    kLogF32,
    kSqrtF32,
    kExpF32,
    kRcpF32,
    kMulHiU32,
    kMadU64U32,
    kBitop3,
    kCvtF32U32,
    kRndneF32,
    kFmaF64,
    kMixSin1Fma3,   // one v_sin_f32 then three v_fma_f32 (4 instructions)
    kMixPair,       // v_sub_f32_dpp, v_sin_f32, two v_add_f32: one coupling pair
    kMixPairNoDpp,  // the same with a plain v_sub_f32
    kMixFolded4,    // one partner phase against four own phases, the read folded into four v_sub_f32_dpp
    kMixMov4,       // the same with one v_mov_b32_dpp and four plain v_sub_f32
    kLibSinF64,
    kLibCosF64,
    kLibLogF64,
    kLibSqrtF64,
    kLibSinF32,     // sinf of the device library (radians, with reduction)
    kPhaseSinF64,   // the coupled kernels' binary64 sine of a phase difference
    kBoxMullerLibF64,  // binary64 Box-Muller pair on the library's log, sqrt, sincospi
    kBoxMullerU24F64,  // the same pair with the 24-bit-uniform log and cos / sin
    kOpCount
};

const char* const kNames[kOpCount] = {
    "v_fma_f32", "v_add_f32", "v_mul_f32", "v_sub_f32_dpp(row_ror)", "v_mov_b32_dpp(row_ror)",
    "v_sin_f32", "v_log_f32", "v_sqrt_f32", "v_exp_f32", "v_rcp_f32", "v_mul_hi_u32",
    "v_mad_u64_u32", "v_bitop3_b32", "v_cvt_f32_u32", "v_rndne_f32", "v_fma_f64",
    "mix: v_sin_f32 + 3 v_fma_f32", "mix: coupling pair (sub_dpp, sin, 2 add)",
    "mix: coupling pair without DPP (sub, sin, 2 add)",
    "mix: 4 pairs, partner read folded (4 sub_dpp, 4 sin, 8 add)",
    "mix: 4 pairs, partner read once (mov_dpp, 4 sub, 4 sin, 8 add)", "binary64 sin (library call)",
    "binary64 cos (library call)", "binary64 log (library call)", "binary64 sqrt (library call)",
    "binary32 sinf (library call)", "binary64 sin_phase64 (coupled kernels' sine, per call)",
    "binary64 Box-Muller pair, library log/sqrt/sincospi (per call)",
    "binary64 Box-Muller pair, 24-bit-uniform log and cos/sin (per call)"};

// Instructions (or library calls) per chain per block.
// Instructions (or library calls) per block of 8 chains.
constexpr double per_block8(int op)
{
    return op == kMixSin1Fma3 || op == kMixPair || op == kMixPairNoDpp ? 32.0
           : op == kMixFolded4                                          ? 32.0
           : op == kMixMov4                                             ? 34.0
                                                                        : 8.0;
}

#define SODE_R8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int OP>
__device__ __forceinline__ void block_f32(float (&a)[kChains], float (&e)[kChains], float b, float c)
{
    if constexpr (OP == kFmaF32) {
#define X(i) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(a[i]) : "v"(b), "v"(c));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kAddF32) {
#define X(i) asm volatile("v_add_f32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kMulF32) {
#define X(i) asm volatile("v_mul_f32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kSubDppF32) {
#define X(i) asm volatile("v_sub_f32_dpp %0, %1, %0 row_ror:1 row_mask:0xf bank_mask:0xf" : "+v"(a[i]) : "v"(b));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kMovDpp) {
#define X(i) asm volatile("v_mov_b32_dpp %0, %1 row_ror:3 row_mask:0xf bank_mask:0xf" : "+v"(a[i]) : "v"(b));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kSinF32) {
#define X(i) asm volatile("v_sin_f32 %0, %0" : "+v"(a[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kLogF32) {
#define X(i) asm volatile("v_log_f32 %0, %0" : "+v"(a[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kSqrtF32) {
#define X(i) asm volatile("v_sqrt_f32 %0, %0" : "+v"(a[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kExpF32) {
#define X(i) asm volatile("v_exp_f32 %0, %0" : "+v"(a[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kRcpF32) {
#define X(i) asm volatile("v_rcp_f32 %0, %0" : "+v"(a[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kCvtF32U32) {
#define X(i) asm volatile("v_cvt_f32_u32 %0, %1" : "+v"(a[i]) : "v"(b));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kRndneF32) {
#define X(i) asm volatile("v_rndne_f32 %0, %0" : "+v"(a[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kMixSin1Fma3) {
        // Sines on a[], fused multiply-adds on e[]: no instruction reads
        // another's result, so only issue limits the rate.
#define X(i)                                                                  \
    asm volatile("v_sin_f32 %0, %0" : "+v"(a[i]));                            \
    asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(e[i]) : "v"(b), "v"(c)); \
    asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(e[(i + 3) % 8]) : "v"(b), "v"(c)); \
    asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(e[(i + 6) % 8]) : "v"(b), "v"(c));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kMixPair || OP == kMixPairNoDpp) {
        // Eight pairs of the pairwise coupling sum, as the coupled kernel
        // issues them: d = other - mine (the partner read folded into the
        // subtraction as a DPP operand), s = sin(d), acc += s, back += s.
        // Phases of eight, so that every result is used eight instructions
        // after it is produced.
        float d[kChains];
#define X(i)                                                                                         \
    if constexpr (OP == kMixPair)                                                                    \
        asm volatile("v_sub_f32_dpp %0, %1, %2 row_ror:5 row_mask:0xf bank_mask:0xf" : "=v"(d[i]) : "v"(b), "v"(a[i])); \
    else                                                                                             \
        asm volatile("v_sub_f32 %0, %1, %2" : "=v"(d[i]) : "v"(b), "v"(a[i]));
        SODE_R8(X)
#undef X
#define X(i) asm volatile("v_sin_f32 %0, %0" : "+v"(d[i]));
        SODE_R8(X)
#undef X
#define X(i) asm volatile("v_add_f32 %0, %1, %0" : "+v"(e[i]) : "v"(d[i]));
        SODE_R8(X)
#undef X
#define X(i) asm volatile("v_add_f32 %0, %1, %0" : "+v"(e[(i + 4) % 8]) : "v"(d[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kMixFolded4 || OP == kMixMov4) {
        // Pairs of one partner phase (read from the lane five rotations
        // away) with the own phases a[0..3], then with a[4..7]: differences,
        // sines, and the two accumulations of each sine, as the 16-lane
        // coupling issues them.
        float d[kChains];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if constexpr (OP == kMixFolded4) {
#define X(i) asm volatile("v_sub_f32_dpp %0, %1, %2 row_ror:5 row_mask:0xf bank_mask:0xf" : "=v"(d[4 * h + i]) : "v"(b), "v"(a[4 * h + i]));
                X(0) X(1) X(2) X(3)
#undef X
            } else {
                float t;
                asm volatile("v_mov_b32_dpp %0, %1 row_ror:5 row_mask:0xf bank_mask:0xf" : "=v"(t) : "v"(b));
#define X(i) asm volatile("v_sub_f32 %0, %1, %2" : "=v"(d[4 * h + i]) : "v"(t), "v"(a[4 * h + i]));
                X(0) X(1) X(2) X(3)
#undef X
            }
#define X(i) asm volatile("v_sin_f32 %0, %0" : "+v"(d[4 * h + i]));
            X(0) X(1) X(2) X(3)
#undef X
#define X(i) asm volatile("v_add_f32 %0, %1, %0" : "+v"(e[4 * h + i]) : "v"(d[4 * h + i]));
            X(0) X(1) X(2) X(3)
#undef X
#define X(i) asm volatile("v_add_f32 %0, %1, %0" : "+v"(e[(4 * h + i + 4) % 8]) : "v"(d[4 * h + i]));
            X(0) X(1) X(2) X(3)
#undef X
        }
    } else if constexpr (OP == kLibSinF32) {
#define X(i) a[i] = sinf(a[i]) + b;
        SODE_R8(X)
#undef X
    }
}

template <int OP>
__device__ __forceinline__ void block_u32(uint32_t (&u)[kChains], uint64_t (&w)[kChains], uint64_t (&cy)[kChains],
                                          uint32_t v)
{
    if constexpr (OP == kMulHiU32) {
#define X(i) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(u[i]) : "v"(v));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kMadU64U32) {
#define X(i) asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[i]), "=s"(cy[i]) : "v"(v), "v"(u[i]));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kBitop3) {
#define X(i) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(u[i]) : "v"(v), "v"(u[(i + 1) % 8]));
        SODE_R8(X)
#undef X
    }
}

template <int OP>
__device__ __forceinline__ void block_f64(double (&x)[kChains], double y)
{
    if constexpr (OP == kFmaF64) {
#define X(i) asm volatile("v_fma_f64 %0, %1, %1, %0" : "+v"(x[i]) : "v"(y));
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kLibSinF64) {
#define X(i) x[i] = sin(x[i]) + y;
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kLibCosF64) {
#define X(i) x[i] = cos(x[i]) + y;
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kLibLogF64) {
#define X(i) x[i] = log(x[i]) + y;
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kLibSqrtF64) {
#define X(i) x[i] = sqrt(x[i]) + y;
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kPhaseSinF64) {
#define X(i) x[i] = sode::sin_phase64(x[i]) + y;
        SODE_R8(X)
#undef X
    } else if constexpr (OP == kBoxMullerLibF64 || OP == kBoxMullerU24F64) {
        // Words from the chain's bits (two integer multiplies and a shift),
        // so every call sees new uniforms; the pair's sum feeds the chain.
#define X(i)                                                                          \
    {                                                                                 \
        const uint64_t bx = __builtin_bit_cast(uint64_t, x[i]);                       \
        const uint32_t wa = (uint32_t)bx * 2654435761u, wb = (uint32_t)(bx >> 20) * 40503u; \
        double zc, zs;                                                                \
        if constexpr (OP == kBoxMullerLibF64)                                         \
            sode::box_muller_f64(wa, wb, zc, zs);                                     \
        else                                                                          \
            sode::box_muller_f64_u24(wa, wb, zc, zs);                                 \
        x[i] = (zc + zs) + y;                                                         \
    }
        SODE_R8(X)
#undef X
    }
}

constexpr bool is_u32(int op) { return op == kMulHiU32 || op == kMadU64U32 || op == kBitop3; }
constexpr bool is_f64(int op)
{
    return op == kFmaF64 || op == kLibSinF64 || op == kLibCosF64 || op == kLibLogF64 || op == kLibSqrtF64 ||
           op == kPhaseSinF64 || op == kBoxMullerLibF64 || op == kBoxMullerU24F64;
}

// out: one float per lane of the grid; stamps: the shader-clock readings
// (start, end) of each wave's loop.  All waves of a workgroup start the loop
// together (after a barrier), so a workgroup's span is the SIMD time its
// waves' instructions took on the CU's four SIMDs.
template <int OP>
__global__ void op_rate_kernel(float* __restrict__ out, unsigned long long* __restrict__ stamps, int iters,
                               float seed)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const float b = seed + 1e-7f * (float)(threadIdx.x & 63);
    const float c = 0.999f;
    float a[kChains], e[kChains];
    uint32_t u[kChains];
    uint64_t w[kChains], cy[kChains];
    double x[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        a[i] = 0.25f + 0.01f * (float)i + b;
        e[i] = 0.5f * a[i];
        cy[i] = 0;
        u[i] = 0x9E3779B9u * (uint32_t)(tid + i);
        w[i] = u[i];
        x[i] = 0.5 + 0.01 * (double)i + (double)b;
    }
    const uint32_t v = 0xD2511F53u ^ (uint32_t)tid;
    const double y = 1e-3 * (double)b;
    __syncthreads();
    const unsigned long long t0 = clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < kRepeat; ++r) {
            if constexpr (is_u32(OP))
                block_u32<OP>(u, w, cy, v);
            else if constexpr (is_f64(OP))
                block_f64<OP>(x, y);
            else
                block_f32<OP>(a, e, b, c);
        }
    }
    const unsigned long long t1 = clock64();
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i)
        acc += a[i] + e[i] + (float)(u[i] ^ (uint32_t)w[i] ^ (uint32_t)(w[i] >> 32) ^ (uint32_t)cy[i]) +
               (float)x[i];
    out[tid] = acc;
    if ((threadIdx.x & 63) == 0) {
        stamps[2 * (tid >> 6)] = t0;
        stamps[2 * (tid >> 6) + 1] = t1;
    }
}

using KernelFn = void (*)(float*, unsigned long long*, int, float);

template <int... I>
struct Table {
    static constexpr KernelFn fns[sizeof...(I)] = {op_rate_kernel<I>...};
};

template <int N, int... I>
struct MakeTable : MakeTable<N - 1, N - 1, I...> {};
template <int... I>
struct MakeTable<0, I...> {
    using type = Table<I...>;
};

using OpTable = MakeTable<kOpCount>::type;

}  // namespace

extern "C" {

int op_rates_count(void) { return kOpCount; }

const char* op_rates_name(int op) { return op >= 0 && op < kOpCount ? kNames[op] : nullptr; }

// Instructions (or library calls) each wave executes for `iters` iterations.
double op_rates_ops_per_wave(int op, int iters)
{
    if (op < 0 || op >= kOpCount)
        return 0.0;
    return (double)iters * kRepeat * per_block8(op);
}

// Run op `op` over `blocks` workgroups of `waves_per_block` waves (4..16, a
// multiple of 4: the same number of waves on each of a CU's four SIMDs).
// Launch one workgroup per CU.  On success: *mean_cycles = mean over
// workgroups of the span of their loops (latest end - earliest start, shader
// clock), *ms = launch duration (HIP events).  Returns 0, or -1 for bad
// arguments, -2 for a HIP error.
int op_rates_run(int op, int blocks, int waves_per_block, int iters, double* mean_cycles, double* ms)
{
    if (op < 0 || op >= kOpCount || blocks < 1 || blocks > (1 << 16) || waves_per_block < 4 ||
        waves_per_block > 16 || waves_per_block % 4 != 0 || iters < 1 || !mean_cycles || !ms)
        return -1;
    const int threads = 64 * waves_per_block;
    const size_t lanes = (size_t)blocks * threads;
    const size_t waves = lanes / 64;
    float* out = nullptr;
    unsigned long long* cyc = nullptr;
    if (hipMalloc(&out, lanes * sizeof(float)) != hipSuccess)
        return -2;
    if (hipMalloc(&cyc, 2 * waves * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipFree(out);
        return -2;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = -2;
    const KernelFn fn = OpTable::fns[op];
    if (rc == 0) {
        // Warm-up launch, then the timed one.
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), 0, nullptr, out, cyc, iters, 0.5f);
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), 0, nullptr, out, cyc, iters, 0.5f);
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            rc = -2;
    }
    if (rc == 0) {
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t;
        unsigned long long* host = new unsigned long long[2 * waves];
        if (hipMemcpy(host, cyc, 2 * waves * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = -2;
        } else {
            double s = 0.0;
            for (int blk = 0; blk < blocks; ++blk) {
                unsigned long long lo = ~0ull, hi = 0;
                for (int wv = 0; wv < waves_per_block; ++wv) {
                    const size_t i = (size_t)blk * waves_per_block + wv;
                    lo = host[2 * i] < lo ? host[2 * i] : lo;
                    hi = host[2 * i + 1] > hi ? host[2 * i + 1] : hi;
                }
                s += (double)(hi - lo);
            }
            *mean_cycles = s / (double)blocks;
        }
        delete[] host;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(cyc);
    return rc;
}

}  // extern "C"
