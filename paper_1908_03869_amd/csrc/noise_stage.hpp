// noise_stage.hpp - the coupled Kuramoto kernels' normals drawn by other
// waves of the workgroup, for ensembles too small to fill the chip.
//
// With few orbits each integrating wave is alone on its SIMD, so a step
// costs the time that wave needs to issue it, and the Philox blocks and
// Box-Muller pairs of its normals are a large part of that.  The normals do
// not depend on the state, so a workgroup can be one integrating wave (G
// orbits of 64/G lanes each, P normals per lane and step) and NW waves that
// draw those orbits' normals a batch of B steps ahead into LDS,
// double-buffered, with one workgroup barrier per batch.  Each normal comes
// from the same Philox block (step, orbit id, j / 4) and the same
// Box-Muller code as when the integrating lanes draw their own, so the
// results are bitwise the same.
//
// Buffer layout: [step of the batch][orbit of the group][normal of the
// orbit] = [t][q][j], NPO = 64 P / G normals per orbit; integrating lane
// L = q (64 / G) + l reads its P normals at [t][L P ...] -- normal j = l P + i
// of orbit q -- contiguous.
#pragma once

#include "launch.hpp"
#include "noise.hpp"
#include "phase64.hpp"

namespace sode {

// Box-Muller pair of the precision: the binary32 one on the transcendental
// unit, or the binary64 one for 24-bit uniforms (the same code as the
// integrating kernels use).
__device__ __forceinline__ void stage_pair(uint32_t a, uint32_t b, float& zc, float& zs)
{
    box_muller_f32(a, b, zc, zs);
}
__device__ __forceinline__ void stage_pair(uint32_t a, uint32_t b, double& zc, double& zs)
{
    box_muller_f64_u24(a, b, zc, zs);
}

// Normals per buffer: 16 KiB of either precision.
constexpr int kStageNormals32 = 4096;
constexpr int kStageNormals64 = 2048;

// Normals of the group's G orbits (o0 .. o0 + G - 1, NPO each per step) for
// the steps of every batch, written by noise wave w (0 .. NW - 1).  Item
// i = (step t, orbit q, block b) of the batch's blocks; lane `lane` of wave
// w takes i = lane + 64 (w + NW m), m = 0, 1, ...: with G NPO / 4 blocks per
// step dividing 64, its orbit q and block b are the same for every m and
// only the step changes.  Args: the kernel's arguments (orbits, stride,
// nsave, seed, orbit_offset, step_offset, ids, seeds).
template <typename R, int STAGE, int G, int NPO, int NW, class Args>
__device__ __forceinline__ void draw_normal_batches(const Args& a, int w, int lane, int64_t o0,
                                                    R (&stage)[2][STAGE], int64_t nbatch)
{
    constexpr int kBlocksPerStep = G * NPO / 4;
    constexpr int B = STAGE / (G * NPO);
    constexpr int kItemsPerLane = kBlocksPerStep * B / (64 * NW);
    static_assert(64 % kBlocksPerStep == 0 && (kBlocksPerStep * B) % (64 * NW) == 0, "noise item mapping");
    const int rem = lane % kBlocksPerStep;
    const int q = rem / (NPO / 4);
    const int b = rem % (NPO / 4);
    // Past the last orbit: the stream of the last one, for lanes that never save.
    const int64_t o = o0 + q < a.orbits ? o0 + q : a.orbits - 1;
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);
    auto draw = [&](int64_t bi) {
        R* __restrict__ dst = stage[bi & 1] + q * NPO + 4 * b;
        const uint32_t k0 = (uint32_t)a.step_offset + (uint32_t)(bi * B);
#pragma unroll 2
        for (int m = 0; m < kItemsPerLane; ++m) {
            const int t = (lane + 64 * (w + NW * m)) / kBlocksPerStep;
            const Block4 wd = philox_4x32_10(k0 + (uint32_t)t, st.oid, (uint32_t)b, 0u, st.key_lo, st.key_hi);
            R z0, z1, z2, z3;
            stage_pair(wd.w0, wd.w1, z0, z1);
            stage_pair(wd.w2, wd.w3, z2, z3);
            R* __restrict__ at = dst + t * (G * NPO);
            at[0] = z0;
            at[1] = z1;
            at[2] = z2;
            at[3] = z3;
        }
    };
    if (nbatch > 0)
        draw(0);
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        __syncthreads();  // matches the integrating wave's barrier before batch bi
        if (bi + 1 < nbatch)
            draw(bi + 1);  // into the buffer batch bi - 1 used, read before this barrier
    }
}

// The integrating wave: f.step(xi) per step with the staged normals and
// f.save(a, s) after every stride-th step (Orbit: the kernel's per-orbit
// state, kNormals = P normals per lane and step).
template <class Orbit, typename R, int STAGE, int G, int NPO, class Args>
__device__ __forceinline__ void integrate_staged(const Args& a, Orbit& f, int lane, const R (&stage)[2][STAGE],
                                                 int64_t nsteps, int64_t nbatch)
{
    constexpr int P = Orbit::kNormals;
    constexpr int B = STAGE / (G * NPO);
    static_assert(G * NPO == 64 * P, "one integrating wave per group");
    f.save(a, 0);
    // Steps left until the next save and the next save's index: the same in
    // every lane (scalar).
    int64_t s = 1, to_save = a.stride;
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        __syncthreads();  // the noise waves have staged batch bi
        const R* __restrict__ src = stage[bi & 1] + lane * P;
        const int64_t k0 = bi * B;
        if (k0 + B <= nsteps) {
            R xi[P];
#pragma unroll
            for (int i = 0; i < P; ++i)
                xi[i] = src[i];
#pragma unroll 4
            for (int t = 0; t < B; ++t) {
                R xn[P];  // read ahead
#pragma unroll
                for (int i = 0; i < P; ++i)
                    xn[i] = src[(t + 1 < B ? t + 1 : t) * (64 * P) + i];
                f.step(xi);
                if (__builtin_expect(--to_save == 0, 0)) {
                    f.save(a, s);
                    ++s;
                    to_save = a.stride;
                }
#pragma unroll
                for (int i = 0; i < P; ++i)
                    xi[i] = xn[i];
            }
        } else {
            for (int t = 0; k0 + t < nsteps; ++t) {
                R xi[P];
#pragma unroll
                for (int i = 0; i < P; ++i)
                    xi[i] = src[t * (64 * P) + i];
                f.step(xi);
                if (__builtin_expect(--to_save == 0, 0)) {
                    f.save(a, s);
                    ++s;
                    to_save = a.stride;
                }
            }
        }
    }
}

// Body of a staged workgroup: wave 0 integrates the group's G orbits, waves
// 1 .. NW draw their normals.  The wave index is uniform in each wave, so
// the branch is scalar and every wave reaches the same number of barriers
// (one per batch).  A row or quad past the last orbit runs (on no input)
// and saves nothing.
template <class Orbit, typename R, int STAGE, int G, int NPO, int NW, class Args>
__device__ __forceinline__ void staged_workgroup(const Args& a, R (&stage)[2][STAGE])
{
    constexpr int B = STAGE / (G * NPO);
    static_assert(G * Orbit::kLanes == 64, "G orbits fill the integrating wave");
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t o0 = (int64_t)blockIdx.x * G;
    const int64_t nsteps = (a.nsave - 1) * a.stride;
    const int64_t nbatch = (nsteps + B - 1) / B;
    if (wave != 0) {
        draw_normal_batches<R, STAGE, G, NPO, NW>(a, wave - 1, lane, o0, stage, nbatch);
        return;
    }
    const int64_t o = o0 + lane / Orbit::kLanes;
    Orbit f(a, o, lane % Orbit::kLanes, o < a.orbits);
    integrate_staged<Orbit, R, STAGE, G, NPO>(a, f, lane, stage, nsteps, nbatch);
}

// Noise waves per integrating wave: the request's choice, or by ensemble
// size.  Up to two integrating waves (groups) per compute unit, two (the
// noise then keeps up with an integrating wave that has a SIMD to itself);
// up to one per SIMD (four per compute unit), one; beyond that none: the
// SIMDs are shared and the waves of other orbits fill each other's gaps, so
// moving the normals to other waves only adds their LDS traffic and barriers.
inline int staged_noise_waves(const Request& r, int64_t groups)
{
    if (r.noise_waves >= 0)
        return r.noise_waves;
    const int cus = device_compute_units();
    return groups <= 2 * (int64_t)cus ? 2 : groups <= 4 * (int64_t)cus ? 1 : 0;
}

}  // namespace sode
