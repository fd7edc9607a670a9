// rnn_mfma.hip - Euler-Maruyama for dense random recurrent networks,
//     dX = (-X + W tanh X + b) dt + sigma dW,
// with the drift's matrix product on the gfx950 matrix cores.  The orbits
// share W (N x N), b and sigma (one parameter row); X is binary32.
//
// Per step the ensemble needs F[o][i] = sum_j W[i][j] tanh(X[o][j]), a GEMM
// of M = N state indices, N' = orbits and K = N.  It is laid out as
// C[i][o] = A[i][j] B[j][o] with A = W and B = tanh(X)^T, so that the
// 32x32 MFMA accumulator of a lane holds, for ONE orbit (o = lane % 32),
// the 16 state indices i = 32 w + 8 (r / 4) + 4 (lane / 32) + r % 4: four
// runs of four consecutive indices.  Each run is exactly one Philox block
// (normals 4b .. 4b+3 of that orbit), so the lane draws its own noise with
// no exchange, and the update X += dt (-X + F + b) + sigma sqrt(dt) xi is
// lane-local.
//
// A workgroup owns 32 orbits and N/32 waves; wave w computes rows
// 32w .. 32w+31 and keeps that slab of W in registers for the whole launch
// (A operands never touch memory again).  tanh(X) goes through LDS,
// double-buffered: each wave writes the new values of its rows into the
// other buffer, one barrier per step, then every wave reads the full
// 32 x N tile as B operands.
//
// GEMM variants:
//   BF16   W and tanh X rounded to bfloat16, fp32 accumulation
//          (v_mfma_f32_32x32x16_bf16, 16 per 32x32 tile-step for N = 256);
//   BF16X3 each operand split as hi + lo in bfloat16, three products
//          hi.hi + hi.lo + lo.hi (Henry, Tang & Heinecke, ARITH 2019),
//          ~2^-16 relative error;
//   FP32   binary32 operands (v_mfma_f32_32x32x2f32).
#include "devmath.hpp"
#include "launch.hpp"
#include "noise.hpp"

#pragma clang fp contract(off)

namespace sode {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kOrbitsPerBlock = 32;
constexpr float kTwoLog2e = 2.88539008177792681472f;  // 2 / ln 2

struct RnnArgs {
    const float* __restrict__ X0;
    const float* __restrict__ p;  // W (N x N row-major), b (N), sigma
    float* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int64_t orbits, stride, nsave;
    float dt, sqdt;
    uint64_t seed, orbit_offset, step_offset;
    int* nonfinite;
};

// tanh(x) = 1 - 2 / (exp(2x) + 1) on the transcendental unit; exact limits
// +-1 for large |x| (exp overflows to inf or underflows to 0).  Absolute
// error ~1e-7.
__device__ __forceinline__ float fast_tanh(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * kTwoLog2e);
    return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);  // 2 r is exact
}

// (hi, lo) bfloat16 pairs of two values: hi = bf16(y), lo = bf16(y - hi),
// with one packed conversion per pair and the widening of hi done on bits.
struct SplitPair {
    uint32_t hi, lo;  // element 0 in bits 15:0, element 1 in bits 31:16
};
__device__ __forceinline__ SplitPair split_bf16(float y0, float y1)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 h = __builtin_convertvector(f32x2{y0, y1}, bf16x2);
    const uint32_t hb = __builtin_bit_cast(uint32_t, h);
    const float r0 = y0 - __builtin_bit_cast(float, hb << 16);
    const float r1 = y1 - __builtin_bit_cast(float, hb & 0xFFFF0000u);
    const bf16x2 l = __builtin_convertvector(f32x2{r0, r1}, bf16x2);
    return SplitPair{hb, __builtin_bit_cast(uint32_t, l)};
}

template <int N, int MODE>
struct Lds {
    // bf16 modes: [buffer][part][orbit][N + 8] (part 1 = lo, BF16X3 only);
    // fp32 mode: [buffer][orbit][2][N/2 + 4] (+4) with j = 2 kk + h stored
    // at [h][kk], so that one 16-byte read yields four consecutive kk.  The
    // paddings keep every 16-byte read aligned and spread the 16 orbits of
    // a read phase over distinct LDS banks.
    static constexpr int kParts = MODE == kRnnBf16x3 ? 2 : 1;
    static constexpr int kPitchBf = N + 8;
    static constexpr int kHalfF = N / 2 + 4;
    static constexpr int kPitchF = 2 * kHalfF + 4;
    static constexpr size_t kBytes =
        MODE == kRnnFp32 ? 2 * kOrbitsPerBlock * kPitchF * sizeof(float)
                         : 2 * kParts * kOrbitsPerBlock * kPitchBf * sizeof(__bf16);
};

template <int N, int MODE>
__global__ __launch_bounds__(64 * (N / 32)) void rnn_mfma_kernel(const RnnArgs a)
{
    using L = Lds<N, MODE>;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int ol = lane & 31;   // orbit within the block (B column / C column)
    const int half = lane >> 5; // k-group of the operands, row offset of C
    const int64_t o = (int64_t)blockIdx.x * kOrbitsPerBlock + ol;
    const bool valid = o < a.orbits;

    const float* __restrict__ W = a.p;
    const float* __restrict__ bias = a.p + (size_t)N * N;
    const float noise_scale = a.p[(size_t)N * N + N] * a.sqdt;
    const int arow = 32 * w + ol;  // row of W this lane feeds as A operand

    // Rows of this lane's 16 state elements.
    int row[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
        row[r] = 32 * w + 8 * (r >> 2) + 4 * half + (r & 3);

    // A operands: the wave's slab of W, resident in registers.
    constexpr int KB = MODE == kRnnFp32 ? N / 2 : N / 16;
    bf16x8 Ah[MODE == kRnnFp32 ? 1 : KB];
    bf16x8 Al[MODE == kRnnBf16x3 ? KB : 1];
    float Af[MODE == kRnnFp32 ? KB : 1];
    if constexpr (MODE == kRnnFp32) {
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
            Af[kk] = W[(size_t)arow * N + 2 * kk + half];
    } else {
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = W[(size_t)arow * N + 16 * kk + 8 * half + e];
                const __bf16 hi = (__bf16)v;
                Ah[kk][e] = hi;
                if constexpr (MODE == kRnnBf16x3)
                    Al[kk][e] = (__bf16)(v - (float)hi);
            }
        }
    }

    float X[16], bv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        X[r] = valid ? a.X0[o * N + row[r]] : 0.0f;
        bv[r] = bias[row[r]];
    }
    float* __restrict__ out_row = a.out + (valid ? o : 0) * a.nsave * N;
    auto save = [&](int64_t s) {
        if (valid) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                note_nonfinite(a.nonfinite, X[r]);
                out_row[s * N + row[r]] = X[r];
            }
        }
    };
    // tanh of the lane's elements into LDS buffer `buf`.
    auto publish = [&](int buf) {
        if constexpr (MODE == kRnnFp32) {
            float* base = reinterpret_cast<float*>(smem) + (size_t)buf * kOrbitsPerBlock * L::kPitchF;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = row[r];
                base[ol * L::kPitchF + (j & 1) * L::kHalfF + (j >> 1)] = fast_tanh(X[r]);
            }
        } else {
            __bf16* base = reinterpret_cast<__bf16*>(smem) + (size_t)buf * L::kParts * kOrbitsPerBlock * L::kPitchBf;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float y[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    y[e] = fast_tanh(X[4 * g + e]);
                if constexpr (MODE == kRnnBf16x3) {
                    const SplitPair a01 = split_bf16(y[0], y[1]);
                    const SplitPair a23 = split_bf16(y[2], y[3]);
                    *reinterpret_cast<uint2*>(base + ol * L::kPitchBf + row[4 * g]) = uint2{a01.hi, a23.hi};
                    *reinterpret_cast<uint2*>(base + (kOrbitsPerBlock + ol) * L::kPitchBf + row[4 * g]) = uint2{a01.lo, a23.lo};
                } else {
                    bf16x4 hi;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        hi[e] = (__bf16)y[e];
                    *reinterpret_cast<bf16x4*>(base + ol * L::kPitchBf + row[4 * g]) = hi;
                }
            }
        }
    };

    const Stream st = orbit_stream(valid ? o : 0, a.seed, a.orbit_offset, valid ? a.ids : nullptr,
                                   valid ? a.seeds : nullptr);
    save(0);
    publish(0);
    __syncthreads();

    int64_t s = 1, next_save = a.stride;
    const int64_t nsteps = (a.nsave - 1) * a.stride;
    for (int64_t k = 0; k < nsteps; ++k) {
        const int cur = (int)(k & 1);
        // Normals of this step: blocks 8 w + 2 g + half of the orbit.
        float xi[16];
        const uint32_t kc = (uint32_t)(a.step_offset + (uint64_t)k);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const Block4 wd = philox_4x32_10(kc, st.oid, (uint32_t)(8 * w + 2 * g + half), 0u, st.key_lo, st.key_hi);
            box_muller_f32(wd.w0, wd.w1, xi[4 * g + 0], xi[4 * g + 1]);
            box_muller_f32(wd.w2, wd.w3, xi[4 * g + 2], xi[4 * g + 3]);
        }
        // F = W tanh(X) for the wave's 32 rows and the block's 32 orbits.
        f32x16 acc = {0};
        if constexpr (MODE == kRnnFp32) {
            const float* base = reinterpret_cast<const float*>(smem) + (size_t)cur * kOrbitsPerBlock * L::kPitchF +
                                ol * L::kPitchF + half * L::kHalfF;
#pragma unroll
            for (int kq = 0; kq < KB; kq += 4) {
                const f32x4 bq = *reinterpret_cast<const f32x4*>(base + kq);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[kq + t], bq[t], acc, 0, 0, 0);
            }
        } else {
            const __bf16* base = reinterpret_cast<const __bf16*>(smem) +
                                 (size_t)cur * L::kParts * kOrbitsPerBlock * L::kPitchBf + ol * L::kPitchBf + 8 * half;
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
                const bf16x8 bh = *reinterpret_cast<const bf16x8*>(base + 16 * kk);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah[kk], bh, acc, 0, 0, 0);
                if constexpr (MODE == kRnnBf16x3) {
                    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(base + kOrbitsPerBlock * L::kPitchBf + 16 * kk);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah[kk], bl, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al[kk], bh, acc, 0, 0, 0);
                }
            }
        }
        // Euler-Maruyama update (Eq. 2) of the lane's 16 elements.
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float f = ((acc[r] - X[r]) + bv[r]);
            X[r] = __builtin_fmaf(noise_scale, xi[r], __builtin_fmaf(f, a.dt, X[r]));
        }
        publish(cur ^ 1);
        if (k + 1 == next_save) {
            save(s);
            ++s;
            next_save += a.stride;
        }
        __syncthreads();
    }
}

template <int N, int MODE>
hipError_t launch_n(const Request& r)
{
    RnnArgs a;
    a.X0 = static_cast<const float*>(r.X0);
    a.p = static_cast<const float*>(r.p);
    a.out = static_cast<float*>(r.out);
    a.ids = r.orbit_ids;
    a.seeds = r.orbit_seeds;
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.dt = (float)r.dt;
    a.sqdt = (float)sqrt(r.dt);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    a.nonfinite = r.nonfinite;
    const size_t lds = Lds<N, MODE>::kBytes;
    auto kern = rnn_mfma_kernel<N, MODE>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    const dim3 grid((unsigned)((r.orbits + kOrbitsPerBlock - 1) / kOrbitsPerBlock));
    hipLaunchKernelGGL(kern, grid, dim3(64 * (N / 32)), lds, r.stream, a);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const Request& r)
{
    switch (r.n) {
    case 64: return launch_n<64, MODE>(r);
    case 128: return launch_n<128, MODE>(r);
    case 256: return launch_n<256, MODE>(r);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool rnn_mfma_supports(int n) { return n == 64 || n == 128 || n == 256; }

hipError_t launch_rnn_mfma_f32(const Request& r, int mode)
{
    switch (mode) {
    case kRnnBf16: return launch_mode<kRnnBf16>(r);
    case kRnnBf16x3: return launch_mode<kRnnBf16x3>(r);
    case kRnnFp32: return launch_mode<kRnnFp32>(r);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sode
