// noise.hpp - device-side Brownian increments for the SDE steppers.
//
// The paper draws uniforms from the Random123 library and turns them into
// standard normals with the Box-Muller transform (Sec. 2.1.2, Eq. 3).  Here
// the generator is Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, the
// paper behind Random123), evaluated statelessly: the block that feeds
// normals 4b..4b+3 of orbit id `oid` at global step k is
//     Philox(counter = (k, oid, b, 0), key = (seed mod 2^32, seed >> 32)),
// so every orbit and step can be regenerated anywhere without stored state.
#pragma once

#ifndef __HIPCC_RTC__  // the run-time compiler provides the HIP runtime itself
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace sode {

struct Block4 {
    uint32_t w0, w1, w2, w3;
};

// Philox-4x32 round structure from the SC'11 paper: the even words are
// multiplied by the two round multipliers, the high halves are mixed with
// the odd words and the round key, and the key advances by the two Weyl
// constants (the golden ratio and sqrt(3) - 1 scaled to 32 bits).
__device__ __forceinline__ Block4 philox_4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t key_lo, uint32_t key_hi)
{
    constexpr uint32_t kMulEven0 = 0xD2511F53u;
    constexpr uint32_t kMulEven2 = 0xCD9E8D57u;
    constexpr uint32_t kWeylLo = 0x9E3779B9u;
    constexpr uint32_t kWeylHi = 0xBB67AE85u;
    // Bit i of the table is the result for input bits (a, b, c) = (i>>2, i>>1, i) & 1.
    constexpr uint32_t kXor3 = 0x96u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // One 32x32 -> 64-bit product per even word (a single v_mad_u64_u32),
        // and one three-input bitwise operation (v_bitop3_b32 with the truth
        // table of a ^ b ^ c) per mixed word.
        const uint64_t p0 = (uint64_t)kMulEven0 * c0;
        const uint64_t p2 = (uint64_t)kMulEven2 * c2;
        c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p2 >> 32), c1, key_lo, kXor3);
        c1 = (uint32_t)p2;
        c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, key_hi, kXor3);
        c3 = (uint32_t)p0;
        key_lo += kWeylLo;
        key_hi += kWeylHi;
    }
    return Block4{c0, c1, c2, c3};
}

// 24-bit uniforms: the first of a pair lies in (0,1] so that its logarithm is
// finite, the second in [0,1).  Both are exact in binary32 and binary64.
__device__ __forceinline__ float unit_open_f32(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }
__device__ __forceinline__ float unit_closed_f32(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ double unit_open_f64(uint32_t w) { return (double)((w >> 8) + 1u) * 0x1p-24; }
__device__ __forceinline__ double unit_closed_f64(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

// Box-Muller pair, Eq. (3): radius sqrt(-2 ln U1), angle 2 pi U2; cosine
// branch first.  Binary32 version on the hardware transcendental unit:
// v_log_f32 returns log2, so -2 ln U1 = -2 ln(2) log2(U1); v_sin/v_cos take
// their argument in revolutions, so U2 is passed as is.
__device__ __forceinline__ void box_muller_f32(uint32_t a, uint32_t b, float& z_cos, float& z_sin)
{
    constexpr float kMinus2Ln2 = -1.38629436111989061883f;
    const float u1 = unit_open_f32(a);
    const float u2 = unit_closed_f32(b);
    const float radius = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u1));
    z_cos = radius * __builtin_amdgcn_cosf(u2);
    z_sin = radius * __builtin_amdgcn_sinf(u2);
}

// Binary64 version on the device math library's functions; sincospi
// takes the half-turn count 2 U2 and avoids rounding 2 pi U2 first.
__device__ __forceinline__ void box_muller_f64(uint32_t a, uint32_t b, double& z_cos, double& z_sin)
{
    const double u1 = unit_open_f64(a);
    const double u2 = unit_closed_f64(b);
    const double radius = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z_cos = radius * c;
    z_sin = radius * s;
}

template <typename R>
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, R& z_cos, R& z_sin);
template <>
__device__ __forceinline__ void box_muller<float>(uint32_t a, uint32_t b, float& zc, float& zs)
{
    box_muller_f32(a, b, zc, zs);
}
template <>
__device__ __forceinline__ void box_muller<double>(uint32_t a, uint32_t b, double& zc, double& zs)
{
    box_muller_f64(a, b, zc, zs);
}

// Noise addressing of one orbit: its id (Philox counter word 1) and its key.
struct Stream {
    uint32_t oid;
    uint32_t key_lo, key_hi;
};

__device__ __forceinline__ Stream orbit_stream(int64_t o, uint64_t seed, uint64_t orbit_offset,
                                               const uint32_t* __restrict__ ids,
                                               const uint64_t* __restrict__ seeds)
{
    Stream s;
    s.oid = ids ? ids[o] : (uint32_t)(orbit_offset + (uint64_t)o);
    const uint64_t sd = seeds ? seeds[o] : seed;
    s.key_lo = (uint32_t)sd;
    s.key_hi = (uint32_t)(sd >> 32);
    return s;
}

// All m normals of one orbit at global step k, written to xi[0..m).
template <typename R>
__device__ __forceinline__ void normals(const Stream& st, uint32_t k, int m, R* xi)
{
    for (int b = 0; 4 * b < m; ++b) {
        const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)b, 0u, st.key_lo, st.key_hi);
        R z0, z1, z2, z3;
        box_muller<R>(w.w0, w.w1, z0, z1);
        box_muller<R>(w.w2, w.w3, z2, z3);
        const int j = 4 * b;
        xi[j] = z0;
        if (j + 1 < m) xi[j + 1] = z1;
        if (j + 2 < m) xi[j + 2] = z2;
        if (j + 3 < m) xi[j + 3] = z3;
    }
}

// Normals P*l .. P*l+P-1 of one orbit at global step k, for a lane l that
// owns P consecutive state components (P = 1..8): the Philox blocks
// floor(P*l/4) .. floor((P*l+P-1)/4).  Lanes with P < 4 and P a power of two
// compute one block and keep their share of it; for P = 3, 5, 6, 7 the
// lane's range starts at word (P*l) mod 4 of its first block and touches at
// most ceil((P+3)/4) blocks, all of which the lane evaluates.
template <int P>
__device__ __forceinline__ void lane_normals(const Stream& st, uint32_t k, int l, float (&xi)[P])
{
    if constexpr (P % 4 == 0) {
#pragma unroll
        for (int g = 0; g < P / 4; ++g) {
            const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)(l * (P / 4) + g), 0u, st.key_lo, st.key_hi);
            box_muller_f32(w.w0, w.w1, xi[4 * g + 0], xi[4 * g + 1]);
            box_muller_f32(w.w2, w.w3, xi[4 * g + 2], xi[4 * g + 3]);
        }
    } else if constexpr (P == 2) {
        const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)(l >> 1), 0u, st.key_lo, st.key_hi);
        const bool upper = (l & 1) != 0;
        box_muller_f32(upper ? w.w2 : w.w0, upper ? w.w3 : w.w1, xi[0], xi[1]);
    } else if constexpr (P == 1) {
        const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)(l >> 2), 0u, st.key_lo, st.key_hi);
        const bool upper = (l & 2) != 0;
        float zc, zs;
        box_muller_f32(upper ? w.w2 : w.w0, upper ? w.w3 : w.w1, zc, zs);
        xi[0] = (l & 1) ? zs : zc;
    } else {
        static_assert(P > 2 && P < 8, "oscillators per lane");
        constexpr int NB = (P + 6) / 4;
        const int j0 = P * l;
        const int off = j0 & 3;
        float z[4 * NB];
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)((j0 >> 2) + g), 0u, st.key_lo, st.key_hi);
            box_muller_f32(w.w0, w.w1, z[4 * g + 0], z[4 * g + 1]);
            box_muller_f32(w.w2, w.w3, z[4 * g + 2], z[4 * g + 3]);
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
            xi[i] = off == 0 ? z[i] : off == 1 ? z[i + 1] : off == 2 ? z[i + 2] : z[i + 3];
    }
}

// Value held by another lane of the same quad of lanes (DPP quad_perm):
// the other lane of an adjacent pair (2m, 2m+1), or lane S of the quad.
__device__ __forceinline__ uint32_t from_pair_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
}
template <int S>
__device__ __forceinline__ float from_quad_lane(float v)
{
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x55 * S, 0xF, 0xF, true));
}

// The normals of lane_normals<P> for the 4/P consecutive steps k .. k+4/P-1
// at once, xi[t] being those of step k+t (P = 1 or 2).  Lanes 4m .. 4m+3
// (P = 1) or 2m, 2m+1 (P = 2) use one Philox block per step between them;
// here each of them evaluates that block for one of the steps and passes
// on the words or normals the others need through DPP, so every block is
// computed once instead of once per lane: the same values, 1/4 or 1/2 of
// the Philox work (and half the Box-Muller work for P = 1).  The lanes of a
// quad must belong to the same orbit and be active together.
template <int P>
__device__ __forceinline__ void lane_normals_steps(const Stream& st, uint32_t k, int l, float (&xi)[4 / P][P])
{
    static_assert(P == 1 || P == 2, "lanes per Philox block");
    if constexpr (P == 2) {
        const bool odd = (l & 1) != 0;
        const Block4 w = philox_4x32_10(k + (odd ? 1u : 0u), st.oid, (uint32_t)(l >> 1), 0u, st.key_lo, st.key_hi);
        // Even lane: block of step k, keeps words 0-1, passes 2-3.  Odd lane:
        // block of step k+1, keeps words 2-3, passes 0-1.
        const uint32_t own0 = odd ? w.w2 : w.w0, own1 = odd ? w.w3 : w.w1;
        const uint32_t got0 = from_pair_lane(odd ? w.w0 : w.w2);
        const uint32_t got1 = from_pair_lane(odd ? w.w1 : w.w3);
        box_muller_f32(odd ? got0 : own0, odd ? got1 : own1, xi[0][0], xi[0][1]);
        box_muller_f32(odd ? own0 : got0, odd ? own1 : got1, xi[1][0], xi[1][1]);
    } else {
        // Lane i of the quad draws all four normals of step k+i; normal j of
        // a step belongs to lane j.
        const int qi = l & 3;
        const Block4 w = philox_4x32_10(k + (uint32_t)qi, st.oid, (uint32_t)(l >> 2), 0u, st.key_lo, st.key_hi);
        float z0, z1, z2, z3;
        box_muller_f32(w.w0, w.w1, z0, z1);
        box_muller_f32(w.w2, w.w3, z2, z3);
        auto mine = [qi](float c0, float c1, float c2, float c3) {
            return (qi & 2) ? ((qi & 1) ? c3 : c2) : ((qi & 1) ? c1 : c0);
        };
        xi[0][0] = mine(from_quad_lane<0>(z0), from_quad_lane<0>(z1), from_quad_lane<0>(z2), from_quad_lane<0>(z3));
        xi[1][0] = mine(from_quad_lane<1>(z0), from_quad_lane<1>(z1), from_quad_lane<1>(z2), from_quad_lane<1>(z3));
        xi[2][0] = mine(from_quad_lane<2>(z0), from_quad_lane<2>(z1), from_quad_lane<2>(z2), from_quad_lane<2>(z3));
        xi[3][0] = mine(from_quad_lane<3>(z0), from_quad_lane<3>(z1), from_quad_lane<3>(z2), from_quad_lane<3>(z3));
    }
}

}  // namespace sode
