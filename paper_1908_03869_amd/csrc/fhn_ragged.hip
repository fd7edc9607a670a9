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
// Noise.  The normals of a step do not depend on the state and are drawn
// ahead of it.  With one or two units per lane, a quad or pair of lanes
// shares each Philox block: lane_normals_steps draws 4 or 2 steps at once,
// every block evaluated by one lane and passed on by DPP.
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
// cost U x steps (longest processing time first).  Waves of the persistent
// grid pop groups with one atomic counter until the list is exhausted, so
// the batch is balanced without knowing in advance which instance finishes
// when.  The wave running a group takes an issue priority (s_setprio) from
// the group's cost relative to the heaviest one, so a critical-path chain
// that shares a SIMD issues first.  The same group body also runs
// non-persistently (one block per group), which gives bitwise the same
// result.
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

template <int L, int U, bool COMP>
__device__ __forceinline__ void run_group(const RaggedKernelArgs& a, int32_t g, int lane)
{
    const int slot = lane / L;
    const int l = lane % L;
    // One instance per wave when L = 64: its descriptor, step count and
    // parameters are then wave-uniform (scalar loads, a uniform loop).
    const int32_t inst = L == 64 ? __builtin_amdgcn_readfirstlane(a.slots[g * kRaggedSlots])
                                 : a.slots[g * kRaggedSlots + slot];
    if (inst < 0)
        return;
    const sode_instance_t d = a.desc[inst];
    const int N = d.n / 2;
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
    auto save = [&](int64_t s) {
        float* __restrict__ row = out + s * d.n;
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
    };
    save(0);
    const Stream st{d.orbit_id, (uint32_t)d.seed, (uint32_t)(d.seed >> 32)};
    int64_t s = 1, next_save = d.stride;
    // One Euler-Maruyama step (Eq. 2) with the normals xi of step k.
    auto advance = [&](int64_t k, const float (&xi)[U]) {
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
        if (k + 1 == next_save) {
            save(s);
            ++s;
            next_save += d.stride;
        }
    };
    // The normals do not depend on the state: they are drawn ahead, off the
    // state's dependency chain.
    if constexpr (U <= 2) {
        // One or two units per lane: the normals of B = 4/U steps at a time,
        // one Philox block per quad (U = 1) or pair (U = 2) of lanes and step
        // (lane_normals_steps), drawn one batch ahead.
        constexpr int B = 4 / U;
        float xc[B][U];
        lane_normals_steps<U>(st, 0u, l, xc);
        for (int64_t k = 0; k < d.nsteps; k += B) {
            float xn[B][U];
            lane_normals_steps<U>(st, (uint32_t)(k + B), l, xn);
#pragma unroll
            for (int t = 0; t < B; ++t) {
                if (t == 0 || k + t < d.nsteps)
                    advance(k + t, xc[t]);
            }
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    xc[t][u] = xn[t][u];
        }
    } else {
        // Normals of step k+1 are drawn while step k's update is in flight.
        float xi_next[U];
        if (d.nsteps > 0)
            lane_normals<U>(st, 0u, l, xi_next);
        for (int64_t k = 0; k < d.nsteps; ++k) {
            float xi[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                xi[u] = xi_next[u];
            if (k + 1 < d.nsteps)
                lane_normals<U>(st, (uint32_t)(k + 1), l, xi_next);
            advance(k, xi);
        }
    }
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
__device__ __forceinline__ void run_shape(const RaggedKernelArgs& a, int32_t g, int lane)
{
    const int32_t word = __builtin_amdgcn_readfirstlane(a.shape[g]);
    set_wave_priority((word >> 8) & 3);
    switch (word & 0xFF) {
    case 0: run_group<4, 1, COMP>(a, g, lane); break;
    case 1: run_group<4, 2, COMP>(a, g, lane); break;
    case 2: run_group<4, 4, COMP>(a, g, lane); break;
    case 3: run_group<4, 8, COMP>(a, g, lane); break;
    case 4: run_group<8, 1, COMP>(a, g, lane); break;
    case 5: run_group<8, 2, COMP>(a, g, lane); break;
    case 6: run_group<8, 4, COMP>(a, g, lane); break;
    case 7: run_group<8, 8, COMP>(a, g, lane); break;
    case 8: run_group<16, 1, COMP>(a, g, lane); break;
    case 9: run_group<16, 2, COMP>(a, g, lane); break;
    case 10: run_group<16, 4, COMP>(a, g, lane); break;
    case 11: run_group<16, 8, COMP>(a, g, lane); break;
    case 12: run_group<32, 1, COMP>(a, g, lane); break;
    case 13: run_group<32, 2, COMP>(a, g, lane); break;
    case 14: run_group<32, 4, COMP>(a, g, lane); break;
    case 15: run_group<32, 8, COMP>(a, g, lane); break;
    case 16: run_group<64, 1, COMP>(a, g, lane); break;
    case 17: run_group<64, 2, COMP>(a, g, lane); break;
    case 18: run_group<64, 4, COMP>(a, g, lane); break;
    case 19: run_group<64, 8, COMP>(a, g, lane); break;
    default: break;
    }
}

__device__ __forceinline__ void run_any(const RaggedKernelArgs& a, int32_t g, int lane)
{
    if (a.compensated)
        run_shape<true>(a, g, lane);
    else
        run_shape<false>(a, g, lane);
}

// Persistent: every wave pops group indices until the list is exhausted
// (an exit every wave reaches).  Lane 0 takes the ticket with a vector
// atomic and the wave reads it back as a uniform value.
__global__ __launch_bounds__(64) void fhn_ragged_persistent(const RaggedKernelArgs a)
{
    const int lane = threadIdx.x;
    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0)
            ticket = atomicAdd(a.counter, 1u);
        const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)ticket);
        if (g >= (uint32_t)a.ngroups)
            break;
        run_any(a, (int32_t)g, lane);
    }
}

// One block per group, no queue: the reference schedule for the tests.
__global__ __launch_bounds__(64) void fhn_ragged_direct(const RaggedKernelArgs a)
{
    run_any(a, (int32_t)blockIdx.x, threadIdx.x);
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
    if (persistent) {
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, stream, a.counter);
        hipLaunchKernelGGL(fhn_ragged_persistent, dim3((unsigned)waves), dim3(64), 0, stream, a);
    } else {
        hipLaunchKernelGGL(fhn_ragged_direct, dim3((unsigned)a.ngroups), dim3(64), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace sode
