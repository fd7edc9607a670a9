// fhn_ragged.hip - one persistent launch for a ragged batch of stochastic
// FitzHugh-Nagumo chains of different sizes and lengths (Euler-Maruyama,
// binary32).  Chain with N units, state (v_1..v_N, w_1..w_N):
//     dv_i = [v_i - v_i^3/3 - w_i + D (v_{i-1} - 2 v_i + v_{i+1})] dt + sigma dW_i
//     dw_i = eps (v_i + a - b w_i) dt,   no-flux ends (v_0 = v_1, v_{N+1} = v_N).
//
// Mapping.  An instance occupies L consecutive lanes (L = 4 .. 64) and each
// lane owns U consecutive units (U = 1, 2, 4 or 8), L * U >= N.  A wave
// therefore carries 64/L instances of the same (L, U) shape.  The only
// cross-lane data is the diffusive coupling of the two units at a lane's
// edges: the left neighbour comes from lane l-1, the right one from lane
// l+1 -- by DPP row_shr:1 / row_shl:1 when an instance fits in a 16-lane
// row, by DPP wave_shr:1 / wave_shl:1 when it spans rows.  Reads
// that cross an instance boundary are never used: they only reach units 0
// and N-1, whose missing neighbour is replaced by the unit itself (no-flux
// ends).  Units with index >= N in the last lanes are computed and never
// stored.  Long chains spread over many lanes keep the per-step dependency
// chain short: a batch cannot finish before its longest instance.
//
// Noise.  The normals of a step do not depend on the state, so they are
// drawn by a second wave of the workgroup, a batch of 32/U steps ahead, and
// staged in LDS (double-buffered, one workgroup barrier per batch).  The
// integrating wave's per-step work is then the drift and the update alone,
// which shortens the dependency chain of every instance: one wave runs its
// steps one after another, so this chain sets how long a long instance takes
// and with it the batch's makespan.  Each normal comes from the Philox block
// (step, orbit id, block j/4) of the stateless counter scheme, so where and
// by which lane it is drawn does not change its value.
//
// Precision.  Near rest the recovery variable moves by ~1e-7 per step,
// below half a binary32 ulp of w ~ 0.6, so plain binary32 updates stall and
// drift over 10^5 steps.  With compensation (the handle's default) v and w
// are carried as hi + lo and every increment is added with Dekker's
// Fast2Sum (exact while the state is at least the increment in magnitude,
// see compensated_add).
//
// Scheduling.  The host groups instances of one shape into groups of 64/L
// (sorted by step count inside a shape) and orders groups by decreasing
// cost U x steps (longest processing time first).  Workgroups of the persistent
// grid pop groups with one atomic counter until the list is exhausted, so
// the batch is balanced without knowing in advance which instance finishes
// when.  Both waves of the workgroup running a group take an issue priority
// (s_setprio) from the group's cost relative to the heaviest one, so a
// critical-path chain that shares a SIMD issues first.  The same group body
// also runs non-persistently (one workgroup per group), which gives bitwise
// the same result.
#include "devmath.hpp"
#include "launch.hpp"
#include "noise.hpp"

#pragma clang fp contract(off)

namespace sode {
namespace {

constexpr float kThird = 1.0f / 3.0f;

template <int CTRL>
__device__ __forceinline__ float dpp_read(float v)
{
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
// row_shr:1 -> value of lane l-1; row_shl:1 -> value of lane l+1 (same row).
__device__ __forceinline__ float from_lower_lane(float v) { return dpp_read<0x111>(v); }
__device__ __forceinline__ float from_upper_lane(float v) { return dpp_read<0x101>(v); }
// wave_shr:1 / wave_shl:1: the same across the whole 64-lane wave (a GFX9
// DPP form), one VALU operation instead of an LDS permute round trip.
__device__ __forceinline__ float from_lower_lane_wave(float v) { return dpp_read<0x138>(v); }
__device__ __forceinline__ float from_upper_lane_wave(float v) { return dpp_read<0x130>(v); }

// x_hi + x_lo += inc, keeping the rounding error of the sum in x_lo:
// Dekker's Fast2Sum of hi and y = inc + lo, exact when |hi| >= |y|.  The
// states here are O(1) and the increments O(dt), so that holds except within
// a few increments of zero, where the error it may leave is below an ulp of
// a sum that small (~1e-9 of the state's scale).  Four operations instead of
// the seven of the branch-free two-sum.
__device__ __forceinline__ void compensated_add(float& hi, float& lo, float inc)
{
    const float y = inc + lo;
    const float s = hi + y;
    lo = y - (s - hi);
    hi = s;
}

// Steps per noise batch for U units per lane: every batch holds
// kBatchNormals normals (64 lanes x U units x B steps), 512 Philox blocks.
template <int U>
constexpr int batch_steps() { return 32 / U; }
constexpr int kBatchNormals = 2048;

// Shared memory of a workgroup: the two halves of the noise stage and the
// queue ticket.  Normal j of the instance in slot s at step t of a batch sits
// at t*64U + s*L*U + j, which is where the integrating wave's lane s*L + j/U
// reads its unit j % U of step t.
struct RaggedShared {
    float stage[2][kBatchNormals];
    int32_t ticket;
};

// Largest step count among the group's instances: the number of steps both
// waves of the workgroup walk through (uniform).
template <int L>
__device__ __forceinline__ int64_t group_steps(const RaggedKernelArgs& a, int32_t g)
{
    int64_t kmax = 0;
#pragma unroll
    for (int s = 0; s < 64 / L; ++s) {
        const int32_t inst = a.slots[g * kRaggedSlots + s];
        if (inst >= 0) {
            const int64_t ns = a.desc[inst].nsteps;
            kmax = ns > kmax ? ns : kmax;
        }
    }
    return kmax;
}

// The noise wave.  Lane p evaluates blocks q = p + 64 i (i < 8) of each
// batch: block q is block r = q mod 16U of step t = q / 16U, i.e. block
// b = r mod (LU/4) of the instance in slot s = r / (LU/4), whose four normals
// 4b .. 4b+3 go to stage[4q .. 4q+3].  The counters are those of the
// one-wave path (step k, instance orbit id, block b), so the values are
// bitwise the same.
template <int L, int U>
__device__ __forceinline__ void produce_noise(const RaggedKernelArgs& a, int32_t g, int lane, RaggedShared& sh,
                                              int64_t kmax)
{
    constexpr int B = batch_steps<U>();
    constexpr int kBlocksPerStep = 16 * U;
    constexpr int kBlocksPerInstance = L * U / 4;
    constexpr int kPerLane = kBatchNormals / 4 / 64;
    uint32_t oid[kPerLane], klo[kPerLane], khi[kPerLane];
    bool ok[kPerLane];
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) {
        const int q = lane + 64 * i;
        const int s = (q % kBlocksPerStep) / kBlocksPerInstance;
        const int32_t inst = a.slots[g * kRaggedSlots + s];
        ok[i] = inst >= 0;
        const sode_instance_t d = a.desc[ok[i] ? inst : 0];
        oid[i] = d.orbit_id;
        klo[i] = (uint32_t)d.seed;
        khi[i] = (uint32_t)(d.seed >> 32);
    }
    auto fill = [&](int64_t k0, float* __restrict__ dst) {
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
            const int q = lane + 64 * i;
            const int t = q / kBlocksPerStep;
            const int b = (q % kBlocksPerStep) % kBlocksPerInstance;
            if (ok[i]) {
                const Block4 w = philox_4x32_10((uint32_t)(k0 + t), oid[i], (uint32_t)b, 0u, klo[i], khi[i]);
                float4 z;
                box_muller_f32(w.w0, w.w1, z.x, z.y);
                box_muller_f32(w.w2, w.w3, z.z, z.w);
                *reinterpret_cast<float4*>(dst + 4 * q) = z;
            }
        }
    };
    const int64_t nbatch = (kmax + B - 1) / B;
    if (nbatch > 0)
        fill(0, sh.stage[0]);
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        __syncthreads();  // batch bi staged; batch bi - 1 consumed
        if (bi + 1 < nbatch)
            fill((bi + 1) * B, sh.stage[(bi + 1) & 1]);
    }
}

// The integrating wave: lanes s*L .. s*L+L-1 step the instance in slot s
// (U units each) with the normals the noise wave staged.
template <int L, int U, bool COMP>
__device__ __forceinline__ void integrate_group(const RaggedKernelArgs& a, int32_t g, int lane, const RaggedShared& sh,
                                                int64_t kmax)
{
    constexpr int B = batch_steps<U>();
    const int slot = lane / L;
    const int l = lane % L;
    // One instance per wave when L = 64: its descriptor, step count, stride
    // and parameters are then wave-uniform (scalar registers), so the step
    // loop's control is scalar.
    const int32_t inst = L == 64 ? __builtin_amdgcn_readfirstlane(a.slots[g * kRaggedSlots])
                                 : a.slots[g * kRaggedSlots + slot];
    // Lanes of an empty slot stay in the loop (the workgroup barrier is
    // reached by every wave) but have no units, no steps and no saves.
    const bool active = inst >= 0;
    const sode_instance_t d = a.desc[active ? inst : 0];
    const int N = active ? d.n / 2 : 0;
    // Step counts and strides are < 2^32 (checked on the host).  The host
    // groups only instances with the same stride, so the save schedule is
    // the same in every lane (saves after steps stride, 2 stride, ...): the
    // stride of slot 0 is taken as a scalar.
    uint32_t nsteps = active ? (uint32_t)d.nsteps : 0u;
    if constexpr (L == 64)
        nsteps = (uint32_t)__builtin_amdgcn_readfirstlane((int)nsteps);
    const uint32_t stride = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.desc[a.slots[g * kRaggedSlots]].stride);
    const float* __restrict__ X0 = a.X0 + d.x0_offset;
    const float* __restrict__ pr = a.p + d.p_offset;
    float* __restrict__ out = a.out + d.out_offset;
    const float pa = pr[0], pb = pr[1], eps = pr[2], D = pr[3];
    const float noise = pr[4] * a.sqdt;
    const float dt = a.dt;
    const float eps_dt = eps * dt;
    // dw = eps dt (v + a - b w) as fma(-b eps dt, w, fma(v, eps dt, a eps dt)).
    const float a_eps_dt = pa * eps_dt, b_eps_dt = pb * eps_dt;

    float v[U], w[U], vlo[U], wlo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = U * l + u;
        v[u] = j < N ? X0[j] : 0.0f;
        w[u] = j < N ? X0[N + j] : 0.0f;
        vlo[u] = 0.0f;
        wlo[u] = 0.0f;
    }
    float* __restrict__ row = out;  // the next save's row
    auto save = [&]() {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = U * l + u;
            if (j < N) {
                note_nonfinite(a.nonfinite, v[u]);
                note_nonfinite(a.nonfinite, w[u]);
                row[j] = v[u];
                row[N + j] = w[u];
            }
        }
        row += d.n;
    };
    save();
    // Steps left until the next save (a save follows the step that brings
    // this to 0); scalar, the same in every lane.
    uint32_t to_save = stride;
    // One Euler-Maruyama step (Eq. 2) with the normals xi.
    auto advance = [&](const float (&xi)[U]) {
        float left_edge, right_edge;
        if constexpr (L <= 16) {
            left_edge = from_lower_lane(v[U - 1]);
            right_edge = from_upper_lane(v[0]);
        } else {
            left_edge = from_lower_lane_wave(v[U - 1]);
            right_edge = from_upper_lane_wave(v[0]);
        }
        float dv[U], dw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = U * l + u;
            float vl = u > 0 ? v[u - 1] : left_edge;
            float vr = u < U - 1 ? v[u + 1] : right_edge;
            vl = j == 0 ? v[u] : vl;
            vr = j == N - 1 ? v[u] : vr;
            const float lap = __builtin_fmaf(-2.0f, v[u], vl) + vr;
            // v - v^3/3 - w as v (1 - v^2/3) - w: four operations with the
            // coupling term instead of six.
            const float shape = __builtin_fmaf(v[u] * v[u], -kThird, 1.0f);
            const float fv = __builtin_fmaf(D, lap, __builtin_fmaf(v[u], shape, -w[u]));
            dv[u] = __builtin_fmaf(noise, xi[u], fv * dt);
            dw[u] = __builtin_fmaf(-b_eps_dt, w[u], __builtin_fmaf(v[u], eps_dt, a_eps_dt));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (COMP) {
                compensated_add(v[u], vlo[u], dv[u]);
                compensated_add(w[u], wlo[u], dw[u]);
            } else {
                v[u] = v[u] + dv[u];
                w[u] = w[u] + dw[u];
            }
        }
    };
    // The lane's normals of step t of the current batch: U consecutive
    // floats.
    auto load_xi = [&](const float* __restrict__ src, int t, float (&xi)[U]) {
        const float* __restrict__ at = src + t * (64 * U) + lane * U;
#pragma unroll
        for (int u = 0; u < U; ++u)
            xi[u] = at[u];
    };
    const uint32_t nbatch = (uint32_t)((kmax + B - 1) / B);
    for (uint32_t bi = 0; bi < nbatch; ++bi) {
        __syncthreads();  // the noise wave has staged batch bi
        const float* __restrict__ src = sh.stage[bi & 1];
        const uint32_t k0 = bi * B;
        // A batch that every active lane runs to its end (the usual case)
        // needs no per-step check of the step count.
        // (A ballot is a scalar value, so this branch and the save counter
        // below stay in scalar control flow.)
        if (__builtin_amdgcn_ballot_w64(active && k0 + B > nsteps) == 0) {
            float xi[U];
            load_xi(src, 0, xi);
#pragma unroll 4
            for (int t = 0; t < B; ++t) {
                float xn[U];
                load_xi(src, t + 1 < B ? t + 1 : t, xn);  // read ahead, off the update's path
                advance(xi);
                if (__builtin_expect(--to_save == 0, 0)) {
                    save();
                    to_save = stride;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    xi[u] = xn[u];
            }
        } else {
            for (int t = 0; t < B; ++t) {
                const bool stepping = k0 + t < nsteps;
                if (stepping) {
                    float xi[U];
                    load_xi(src, t, xi);
                    advance(xi);
                }
                if (--to_save == 0) {
                    // An instance that has finished saved its last state at
                    // its final step (a multiple of the stride).
                    if (stepping)
                        save();
                    to_save = stride;
                }
            }
        }
    }
}

// A group on a two-wave workgroup: wave 0 integrates, wave 1 draws the
// noise a batch ahead.  The normals do not depend on the state, so taking
// them off the integrating wave shortens the per-step dependency chain of
// every instance to its drift and update: a batch cannot finish before its
// longest instance, which that chain bounds.
template <int L, int U, bool COMP>
__device__ __forceinline__ void run_group(const RaggedKernelArgs& a, int32_t g, int wave, int lane, RaggedShared& sh)
{
    // Uniform by construction (same loads in every lane); made explicit so
    // the batch loops, and the barriers in them, are scalar control flow.
    const int64_t km = group_steps<L>(a, g);
    const int64_t kmax = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(km >> 32)) << 32) |
                                   (uint32_t)__builtin_amdgcn_readfirstlane((int)km));
    if (wave == 0)
        integrate_group<L, U, COMP>(a, g, lane, sh, kmax);
    else
        produce_noise<L, U>(a, g, lane, sh, kmax);
}

// Issue priority of the wave among the waves of its SIMD (s_setprio takes
// an immediate).
__device__ __forceinline__ void set_wave_priority(int p)
{
    if (p >= 3)
        __builtin_amdgcn_s_setprio(3);
    else if (p == 2)
        __builtin_amdgcn_s_setprio(2);
    else if (p == 1)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// Shape word of a group: shape code in bits 0-7, issue priority in bits 8-9.
template <bool COMP>
__device__ __forceinline__ void run_shape(const RaggedKernelArgs& a, int32_t g, int wave, int lane, RaggedShared& sh)
{
    const int32_t word = __builtin_amdgcn_readfirstlane(a.shape[g]);
    set_wave_priority((word >> 8) & 3);
    switch (word & 0xFF) {
    case 0: run_group<4, 1, COMP>(a, g, wave, lane, sh); break;
    case 1: run_group<4, 2, COMP>(a, g, wave, lane, sh); break;
    case 2: run_group<4, 4, COMP>(a, g, wave, lane, sh); break;
    case 3: run_group<4, 8, COMP>(a, g, wave, lane, sh); break;
    case 4: run_group<8, 1, COMP>(a, g, wave, lane, sh); break;
    case 5: run_group<8, 2, COMP>(a, g, wave, lane, sh); break;
    case 6: run_group<8, 4, COMP>(a, g, wave, lane, sh); break;
    case 7: run_group<8, 8, COMP>(a, g, wave, lane, sh); break;
    case 8: run_group<16, 1, COMP>(a, g, wave, lane, sh); break;
    case 9: run_group<16, 2, COMP>(a, g, wave, lane, sh); break;
    case 10: run_group<16, 4, COMP>(a, g, wave, lane, sh); break;
    case 11: run_group<16, 8, COMP>(a, g, wave, lane, sh); break;
    case 12: run_group<32, 1, COMP>(a, g, wave, lane, sh); break;
    case 13: run_group<32, 2, COMP>(a, g, wave, lane, sh); break;
    case 14: run_group<32, 4, COMP>(a, g, wave, lane, sh); break;
    case 15: run_group<32, 8, COMP>(a, g, wave, lane, sh); break;
    case 16: run_group<64, 1, COMP>(a, g, wave, lane, sh); break;
    case 17: run_group<64, 2, COMP>(a, g, wave, lane, sh); break;
    case 18: run_group<64, 4, COMP>(a, g, wave, lane, sh); break;
    case 19: run_group<64, 8, COMP>(a, g, wave, lane, sh); break;
    default: break;
    }
}

__device__ __forceinline__ void run_any(const RaggedKernelArgs& a, int32_t g, int wave, int lane, RaggedShared& sh)
{
    if (a.compensated)
        run_shape<true>(a, g, wave, lane, sh);
    else
        run_shape<false>(a, g, wave, lane, sh);
}

// Persistent: workgroup b first runs group b, then pops group indices
// gridDim.x, gridDim.x + 1, ... until the list is exhausted (an exit both
// waves reach: they read the same ticket).  Thread 0 takes the ticket with a
// vector atomic and publishes it through LDS.  The static first pass hands
// the heaviest groups (the list is in decreasing cost) to consecutive
// workgroups, which the dispatcher spreads over the chip; popped from the
// queue, they went to whichever workgroups reached the counter first, often
// neighbours on one compute unit, and the batch took 10.6-12.3 ms instead
// of 10.4-10.7 ms from one launch to the next.
__global__ __launch_bounds__(128) void fhn_ragged_persistent(const RaggedKernelArgs a)
{
    __shared__ RaggedShared sh;
    // The wave index is uniform in each wave: a scalar value, so the
    // integrate / noise branch is a scalar branch.
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    for (uint32_t pass = 0;; ++pass) {
        uint32_t g = blockIdx.x;
        if (pass > 0) {
            if (threadIdx.x == 0)
                sh.ticket = (int32_t)(gridDim.x + atomicAdd(a.counter, 1u));
            __syncthreads();
            g = (uint32_t)__builtin_amdgcn_readfirstlane(sh.ticket);
            __syncthreads();  // both waves hold the ticket before it is replaced
        }
        if (g >= (uint32_t)a.ngroups)
            break;
        // The lane index passes through an empty asm statement on every
        // pass, so the compiler does not hoist the lane-dependent set-up of
        // all forty group variants out of this loop (that kept it live for
        // the whole kernel and more than doubled the register count); the
        // mask restores what it knows of its range.
        int lane_g = lane;
        asm volatile("" : "+v"(lane_g));
        run_any(a, (int32_t)g, wave, lane_g & 63, sh);
    }
}

// One workgroup per group, no queue: the reference schedule for the tests.
__global__ __launch_bounds__(128) void fhn_ragged_direct(const RaggedKernelArgs a)
{
    __shared__ RaggedShared sh;
    run_any(a, (int32_t)blockIdx.x, __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), threadIdx.x & 63, sh);
}

__global__ void reset_counter(uint32_t* c)
{
    if (threadIdx.x == 0)
        *c = 0u;
}

}  // namespace

int ragged_shape_code(int lanes, int units)
{
    const int li = lanes == 4 ? 0 : lanes == 8 ? 1 : lanes == 16 ? 2 : lanes == 32 ? 3 : 4;
    const int ui = units == 1 ? 0 : units == 2 ? 1 : units == 4 ? 2 : 3;
    return li * 4 + ui;
}

hipError_t launch_fhn_ragged(const RaggedKernelArgs& a, int persistent, int waves, hipStream_t stream)
{
    if (a.ngroups <= 0)
        return hipSuccess;
    // Two waves per workgroup (integration and noise), so `waves` waves are
    // waves / 2 workgroups.
    if (persistent) {
        const unsigned blocks = (unsigned)(waves > 2 ? waves / 2 : 1);
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, stream, a.counter);
        hipLaunchKernelGGL(fhn_ragged_persistent, dim3(blocks), dim3(128), 0, stream, a);
    } else {
        hipLaunchKernelGGL(fhn_ragged_direct, dim3((unsigned)a.ngroups), dim3(128), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace sode
