// kuramoto_lanes.hpp - device building blocks shared by the binary32
// Kuramoto kernels that map one orbit to a 16-lane DPP row (integration,
// checkpointed forward pass and adjoint).  All of them step through
// em_step(), so a recomputed segment reproduces the forward pass bit for bit.
//
// Lane l of a row owns the P = N/16 consecutive oscillators P*l .. P*l+P-1.
// The state is kept in radians, wrapped to [-pi, pi] after every step with a
// two-constant 2 pi reduction (no rounding when no wrap occurs).  With
// compensation off the saved phases are the state itself, so a saved state
// fed back in resumes bit-exactly.  With compensation on each phase is an
// unevaluated sum hi + lo: the rounding error of every update is carried in
// lo (Fast2Sum, exact away from zero), so rounding no longer random-walks
// the binary32 trajectory by ~1e-7 rad per step; saves and checkpoints hold
// hi, and the checkpointed forward pass restarts lo at 0 after each
// checkpoint, so the adjoint's recomputation from a checkpoint matches it.
// Once per step each phase is scaled to revolutions, the argument unit of
// the hardware v_sin_f32, which then evaluates sin(theta_j - theta_i)
// straight from the difference of two scaled phases.
//
// Coupling sum S_i = sum_j sin(theta_j - theta_i).  The paper's loop (Fig. 5)
// evaluates all N^2 sines; here every unordered pair {i, j} is evaluated
// once and used twice, since sin(theta_i - theta_j) = -sin(theta_j - theta_i)
// exactly in IEEE arithmetic (the difference and the sine are both odd
// under negation) and the j = i term is sin(0) = 0.  Pairs inside a lane
// use registers; a pair between lane l and lane l' = l (+/-) k (k = 1..7)
// is evaluated by one of the two lanes, which reads the partner's phases
// with a DPP row rotation and returns the negated partial sums with the
// inverse rotation.  For k = 8 (the opposite lane, a rotation that is its
// own inverse) lane l evaluates its oscillator a against the partner's b for
// a < b only, the partner covering a > b the same way, and both lanes
// evaluate a = b, each for its own side.  Per orbit-step this is
// N(N-1)/2 + N/2 = N^2/2 sines instead of N^2.
//
// Noise: lane l needs normals P*l .. P*l+P-1 (lane_normals, noise.hpp).
//
// Padding (PAD): a system of N oscillators with N not a multiple of 16 runs
// as 16P = 16 ceil(N/16) oscillators, the Q = 16P - N extra ones held at
// phase 0 with zero frequency, coupling and noise coefficients, so they never
// move.  Each pad adds sin(0 - theta_i) to a real oscillator's sum; adding
// Q sin(theta_i) back once per step removes it (exact in real arithmetic,
// one sine per oscillator instead of a mask per pair).  Mean-field sums and
// the order parameter weight pads by 0 and divide by N.
#pragma once

#include "noise.hpp"

// Every product and sum below rounds as written; fused multiply-adds appear
// only where spelled out, so the arithmetic does not depend on the kernel the
// code is inlined into.
#pragma clang fp contract(off)

namespace sode {
namespace kuramoto {

constexpr float kInvTwoPi = 0.159154943091895335768883763373f;
// 2 pi as its binary32 value plus the binary32 remainder.  The reduction
// theta - k head - k tail with fused multiply-adds leaves theta untouched
// when k = 0 (no wrap this step) and otherwise rounds twice.
constexpr float kTwoPiHead = 6.28318548202514648437500f;
constexpr float kTwoPiTail = -1.74845553146951715461e-07f;
constexpr float kPiF = 3.14159274101257324219f;  // binary32 pi, just above pi

// Value of `v` held by another lane of the same 16-lane row, selected by a
// DPP row rotation (control 0x120 + r, r = 1..15).  A rotation has no
// invalid source lane, so bound_ctrl is set only to tell the compiler that
// the old destination value is never used (no register is cleared for it).
template <int R>
__device__ __forceinline__ float row_rotate(float v)
{
    static_assert(R >= 1 && R <= 15, "row rotation amount");
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x120 + R, 0xF, 0xF, true));
}

__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
// theta reduced to [-pi, pi]: theta - 2 pi rint(theta / 2 pi).
__device__ __forceinline__ float wrap_rad(float x)
{
    const float k = __builtin_rintf(x * kInvTwoPi);
    x = __builtin_fmaf(-k, kTwoPiHead, x);
    return __builtin_fmaf(-k, kTwoPiTail, x);
}

// Partner phases from LDS (the LDS form of the coupling sums): each lane
// stores its P scaled phases once per step at row + P l, and reads the P
// phases of lane (l + K) mod 16 -- the lane row_rotate<16 - K> reads -- with
// one or two vector loads instead of P subtractions that each carry a DPP
// operand.  The values, and so the results, are those of the DPP form.
template <int P>
__device__ __forceinline__ void lds_store_phases(float* row, int l, const float (&phi)[P])
{
    if constexpr (P % 4 == 0) {
#pragma unroll
        for (int g = 0; g < P / 4; ++g)
            reinterpret_cast<float4*>(row + P * l)[g] = make_float4(phi[4 * g], phi[4 * g + 1], phi[4 * g + 2], phi[4 * g + 3]);
    } else if constexpr (P == 2) {
        *reinterpret_cast<float2*>(row + 2 * l) = make_float2(phi[0], phi[1]);
    } else {
#pragma unroll
        for (int i = 0; i < P; ++i)
            row[P * l + i] = phi[i];
    }
}

template <int P>
__device__ __forceinline__ void lds_load_phases(const float* row, int lane, float (&out)[P])
{
    if constexpr (P % 4 == 0) {
#pragma unroll
        for (int g = 0; g < P / 4; ++g) {
            const float4 v = reinterpret_cast<const float4*>(row + P * lane)[g];
            out[4 * g] = v.x;
            out[4 * g + 1] = v.y;
            out[4 * g + 2] = v.z;
            out[4 * g + 3] = v.w;
        }
    } else if constexpr (P == 2) {
        const float2 v = *reinterpret_cast<const float2*>(row + 2 * lane);
        out[0] = v.x;
        out[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < P; ++i)
            out[i] = row[P * lane + i];
    }
}

// Rows whose pairwise step reads the partner phases from LDS: 2, 4 or 8
// oscillators per lane (one or two vector loads per partner lane).  With 3,
// 5, 6 or 7 the loads are scalar and the DPP form is as fast or faster.
template <int P, bool MF>
constexpr bool kLdsPartnerPhases = !MF && (P == 2 || P == 4 || P == 8);

// Orders one wave's LDS accesses across its lanes: stores before the loads
// that follow, loads before the stores that follow.  The LDS serves a
// wave's operations in order, so this emits no wait; it keeps the compiler
// from moving the accesses across each other.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pairs between this lane and the lane K rotations away (K = 1..7); LDS:
// partner phases from the row's copy in LDS (row), else by DPP.
template <int P, int K, bool LDS>
__device__ __forceinline__ void couple_across(const float (&phi)[P], float (&acc)[P], const float* row, int l)
{
    float back[P], other[P];
    if constexpr (LDS)
        lds_load_phases<P>(row, (l + K) & 15, other);
    // DPP form: partner phase b, then its P uses right after it: the
    // compiler folds a DPP move into its uses (v_sub_f32_dpp) only when they
    // follow within a few instructions.  Every sum still takes its terms in
    // the same order (acc[a] over b, back[b] over a).  back[b] starts from its
    // first term (0 + s is not an identity under IEEE signed zeros, so a zero
    // start would cost an add per b).
#pragma unroll
    for (int b = 0; b < P; ++b) {
        if constexpr (!LDS)
            other[b] = row_rotate<16 - K>(phi[b]);
#pragma unroll
        for (int a = 0; a < P; ++a) {
            const float s = sin_rev(other[b] - phi[a]);
            acc[a] += s;
            back[b] = a == 0 ? s : back[b] + s;
        }
    }
#pragma unroll
    for (int b = 0; b < P; ++b)
        acc[b] -= row_rotate<K>(back[b]);
}

// Rotations K .. 7 below LIM.
template <int P, int K, bool LDS, int LIM>
__device__ __forceinline__ void couple_rotations(const float (&phi)[P], float (&acc)[P], const float* row, int l)
{
    if constexpr (K <= 7 && K < LIM) {
        couple_across<P, K, LDS>(phi, acc, row, l);
        couple_rotations<P, K + 1, LDS, LIM>(phi, acc, row, l);
    }
}

// LDS: partner phases through row (16 P floats of LDS for this lane's row,
// aligned to 16 bytes), else by DPP row rotations.  LIM <= 8: only the
// rotations below LIM and not the opposite lane (short rows, see
// lane_coefficients).
template <int P, bool LDS = false, int LIM = 9>
__device__ __forceinline__ void coupling_sums(const float (&phi)[P], float (&acc)[P], float* row = nullptr,
                                              int l = 0)
{
    if constexpr (LDS) {
        lds_store_phases<P>(row, l, phi);
        wave_lds_sync();
    }
    // Pairs inside the lane.  Each sum starts from its first term (with
    // P = 1 there is none and the sums start at 0); the pair order and thus
    // the rounding are those of a zero start.
    if constexpr (P == 1) {
        acc[0] = 0.0f;
    } else {
#pragma unroll
        for (int a = 0; a < P; ++a) {
#pragma unroll
            for (int b = a + 1; b < P; ++b) {
                const float s = sin_rev(phi[b] - phi[a]);
                // In this order every sum's first term comes from the pair
                // (0, b): acc[0] from (0, 1), acc[b] from (0, b).
                acc[a] = (a == 0 && b == 1) ? s : acc[a] + s;
                acc[b] = a == 0 ? -s : acc[b] - s;
            }
        }
    }
    couple_rotations<P, 1, LDS, LIM>(phi, acc, row, l);
    if constexpr (LIM <= 8)
        return;
    // Opposite lane (rotation by 8 is its own inverse).  Pairs (own a,
    // partner b) with a < b are evaluated here and returned to the partner,
    // whose own evaluation covers a > b; a == b (the partner's oscillator of
    // the same index) is evaluated by both lanes, each for its own side.
    float back[P], other[P];
    if constexpr (LDS) {
        lds_load_phases<P>(row, (l + 8) & 15, other);
        wave_lds_sync();  // every lane's loads before the next step's stores
    }
#pragma unroll
    for (int b = 0; b < P; ++b) {
        if constexpr (!LDS)
            other[b] = row_rotate<8>(phi[b]);
#pragma unroll
        for (int a = 0; a <= b; ++a) {
            const float s = sin_rev(other[b] - phi[a]);
            acc[a] += s;
            if (a < b)
                back[b] = a == 0 ? s : back[b] + s;
        }
    }
#pragma unroll
    for (int b = 1; b < P; ++b)
        acc[b] -= row_rotate<8>(back[b]);
}

// Sum over the 16 lanes of a row; every lane receives the total.
__device__ __forceinline__ float row_sum(float v)
{
    v += row_rotate<8>(v);
    v += row_rotate<4>(v);
    v += row_rotate<2>(v);
    v += row_rotate<1>(v);
    return v;
}

// Per-lane constants of the Euler-Maruyama map in radians: omega_i dt,
// p_i sqrt(dt) and K dt / N; with padding, K dt / N and a weight per
// oscillator (0 for pads) and the pad count Q.
template <int P, bool PAD = false>
struct LaneCoefficients {
    float drift0[P];
    float noise_scale[P];
    float kc[PAD ? P : 1];
    float weight[PAD ? P : 1];
    float pads;
};

// p = (K, omega_1..N, p_1..N) of the N-oscillator system (N = n_real).
// short_row: one oscillator per lane, N <= 8, coupling sums over the
// rotations below N only (coupling_sums with LIM = N): lanes N .. 15 are
// pads, the rotations by N .. 7 and by 8 pair real lanes with pads only,
// and every real lane meets N - 1 pads (i through its own rotations,
// N - 1 - i through the pads' returns) instead of 16 - N.
template <int P, bool PAD = false>
__device__ __forceinline__ LaneCoefficients<P, PAD> lane_coefficients(const float* __restrict__ p, int l,
                                                                      float dt, float sqdt, float dt_over_n,
                                                                      int n_real = 16 * P, bool short_row = false)
{
    LaneCoefficients<P, PAD> c;
    const float kc = p[0] * dt_over_n;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int osc = P * l + i;
        const bool real = !PAD || osc < n_real;
        c.drift0[i] = real ? p[1 + osc] * dt : 0.0f;
        c.noise_scale[i] = real ? p[1 + n_real + osc] * sqdt : 0.0f;
        if constexpr (PAD) {
            c.kc[i] = real ? kc : 0.0f;
            c.weight[i] = real ? 1.0f : 0.0f;
        }
    }
    if constexpr (!PAD)
        c.kc[0] = kc;
    c.pads = (float)(short_row ? n_real - 1 : 16 * P - n_real);
    return c;
}

// Phase of an initial or checkpointed state.  A value already in range is
// taken as is, so a saved state passed back in continues bit-exactly.
__device__ __forceinline__ float load_phase(float x) { return __builtin_fabsf(x) <= kPiF ? x : wrap_rad(x); }

// Coupling sums through the angle-difference identity:
// sum_j sin(theta_j - theta_i) = cos(theta_i) S - sin(theta_i) C with the row
// sums C = sum cos, S = sum sin -- O(N) per orbit instead of N(N-1)/2 sines.
template <int P, bool PAD>
__device__ __forceinline__ void mean_field_sums(const float (&phi)[P], float (&acc)[P],
                                                const LaneCoefficients<P, PAD>& co)
{
    float cs[P], sn[P], c = 0.0f, s = 0.0f;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        cs[i] = cos_rev(phi[i]);
        sn[i] = sin_rev(phi[i]);
        if constexpr (PAD) {
            c += cs[i] * co.weight[i];
            s += sn[i] * co.weight[i];
        } else {
            c += cs[i];
            s += sn[i];
        }
    }
    const float C = row_sum(c), S = row_sum(s);
#pragma unroll
    for (int i = 0; i < P; ++i)
        acc[i] = cs[i] * S - sn[i] * C;
}

// One Euler-Maruyama step (Eq. 6) of the lane's P oscillators at global
// step k: theta += omega dt + (K/N) S dt + p sqrt(dt) xi, then wrap.
// COMP: th is the leading part of hi + lo and tl the trailing part; the
// increment and the old trailing part are added with a compensated sum
// (Fast2Sum), and a wrap moves the tail of 2 pi into tl.  MF: coupling through the
// mean-field identity instead of pairwise sines.  PAD: see the top of the file.
// xi_out (optional) receives the step's P normals; xi_in (optional) supplies
// them, already drawn (lane_normals_steps), instead of lane_normals.  LDS:
// pairwise partner phases through `row` (coupling_sums); the same results.
template <int P, bool COMP, bool MF = false, bool PAD = false, bool LDS = false, int LIM = 9>
__device__ __forceinline__ void em_step(float (&th)[P], float (&tl)[P], const LaneCoefficients<P, PAD>& c,
                                        const Stream& st, uint32_t k, int l, float* xi_out = nullptr,
                                        const float* xi_in = nullptr, float* row = nullptr)
{
    float phi[P], acc[P], xi[P];
#pragma unroll
    for (int i = 0; i < P; ++i)
        phi[i] = th[i] * kInvTwoPi;
    if constexpr (MF) {
        mean_field_sums<P, PAD>(phi, acc, c);
    } else {
        coupling_sums<P, LDS, LIM>(phi, acc, row, l);
        if constexpr (PAD) {
#pragma unroll
            for (int i = 0; i < P; ++i)
                acc[i] = __builtin_fmaf(c.pads, sin_rev(phi[i]), acc[i]);
        }
    }
    if (xi_in) {
#pragma unroll
        for (int i = 0; i < P; ++i)
            xi[i] = xi_in[i];
    } else {
        lane_normals<P>(st, k, l, xi);
    }
    if (xi_out) {  // the step's normals, for a caller that needs them again
#pragma unroll
        for (int i = 0; i < P; ++i)
            xi_out[i] = xi[i];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const float kc = PAD ? c.kc[i] : c.kc[0];
        const float inc = __builtin_fmaf(c.noise_scale[i], xi[i], __builtin_fmaf(kc, acc[i], c.drift0[i]));
        if constexpr (COMP) {
            // Dekker's Fast2Sum of th and y: exact when |th| >= |y|.  Phases
            // are O(1) and increments O(dt), so that holds except within a
            // few increments of zero, where what it may leave out is below
            // an ulp of a sum that small.
            const float y = inc + tl[i];
            const float s = th[i] + y;
            const float err = y - (s - th[i]);
            const float kw = __builtin_rintf(s * kInvTwoPi);
            th[i] = __builtin_fmaf(-kw, kTwoPiHead, s);
            tl[i] = __builtin_fmaf(-kw, kTwoPiTail, err);
        } else {
            th[i] = wrap_rad(th[i] + inc);
        }
    }
}

// Row sums of cos(theta) and sin(theta) (every lane of the row gets them).
template <int P>
__device__ __forceinline__ void phase_sums(const float (&th)[P], float (&cs)[P], float (&sn)[P], float& C, float& S)
{
    float c = 0.0f, s = 0.0f;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const float rev = th[q] * kInvTwoPi;
        cs[q] = cos_rev(rev);
        sn[q] = sin_rev(rev);
        c += cs[q];
        s += sn[q];
    }
    C = row_sum(c);
    S = row_sum(s);
}

// Order parameter of Eq. (7): r = |sum_j e^{i theta_j}| / N.
template <int P>
__device__ __forceinline__ float order_parameter(const float (&th)[P])
{
    float cs[P], sn[P], C, S;
    phase_sums<P>(th, cs, sn, C, S);
    return __builtin_sqrtf(C * C + S * S) * (1.0f / (float)(16 * P));
}

// The same over the N real oscillators of a padded row (weights 0 for pads).
template <int P>
__device__ __forceinline__ float order_parameter_padded(const float (&th)[P], const float (&weight)[P], float inv_n)
{
    float c = 0.0f, s = 0.0f;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const float rev = th[q] * kInvTwoPi;
        c += cos_rev(rev) * weight[q];
        s += sin_rev(rev) * weight[q];
    }
    const float C = row_sum(c), S = row_sum(s);
    return __builtin_sqrtf(C * C + S * S) * inv_n;
}

}  // namespace kuramoto
}  // namespace sode
