// kuramoto_coupled.hip - binary32 Euler-Maruyama for the stochastic Kuramoto
// network (Eq. 5/6 of Sec. 2.2.1) with all-to-all sine coupling.
//
// Mapping on gfx950: one orbit per DPP row (16 lanes), four orbits per wave.
// Lane l of a row owns the P = N/16 consecutive oscillators P*l .. P*l+P-1.
// The state is kept in radians, wrapped to [-pi, pi] after every step with a
// two-constant 2 pi reduction (exact when no wrap occurs), so saved phases
// are the state itself and a saved state fed back in resumes bit-exactly.
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
// inverse rotation; for k = 8 both lanes evaluate their own side.  Per
// orbit-step this is N(N-1)/2 + N^2/32 sines instead of N^2.
//
// Noise: lane l needs normals P*l .. P*l+P-1, i.e. Philox blocks
// floor(P*l/4) .. floor((P*l+P-1)/4) of its orbit (Sec. 2.1.2).
#include "launch.hpp"
#include "noise.hpp"

namespace sode {
namespace {

constexpr float kInvTwoPi = 0.159154943091895335768883763373f;
// 2 pi as its binary32 value plus the binary32 remainder.  The reduction
// theta - k head - k tail with fused multiply-adds leaves theta untouched
// when k = 0 (no wrap this step) and otherwise rounds twice.
constexpr float kTwoPiHead = 6.28318548202514648437500f;
constexpr float kTwoPiTail = -1.74845553146951715461e-07f;
constexpr float kPiF = 3.14159274101257324219f;  // binary32 pi, just above pi

struct CoupledArgs {
    const float* __restrict__ X0;
    const float* __restrict__ p;
    float* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int p_per_orbit, observable;
    int64_t orbits, stride, nsave;
    float dt;           // dt
    float sqdt;         // sqrt(dt)
    float coupling_dt;  // dt / N
    uint64_t seed, orbit_offset, step_offset;
};

// Value of `v` held by another lane of the same 16-lane row, selected by a
// DPP row rotation (control 0x120 + r, r = 1..15).
template <int R>
__device__ __forceinline__ float row_rotate(float v)
{
    static_assert(R >= 1 && R <= 15, "row rotation amount");
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x120 + R, 0xF, 0xF, false));
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

// Pairs between this lane and the lane K rotations away (K = 1..7).
template <int P, int K>
__device__ __forceinline__ void couple_across(const float (&phi)[P], float (&acc)[P])
{
    float other[P], back[P];
#pragma unroll
    for (int b = 0; b < P; ++b) {
        other[b] = row_rotate<16 - K>(phi[b]);
        back[b] = 0.0f;
    }
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int b = 0; b < P; ++b) {
            const float s = sin_rev(other[b] - phi[a]);
            acc[a] += s;
            back[b] += s;
        }
    }
#pragma unroll
    for (int b = 0; b < P; ++b)
        acc[b] -= row_rotate<K>(back[b]);
}

template <int P, int K>
__device__ __forceinline__ void couple_rotations(const float (&phi)[P], float (&acc)[P])
{
    if constexpr (K <= 7) {
        couple_across<P, K>(phi, acc);
        couple_rotations<P, K + 1>(phi, acc);
    }
}

template <int P>
__device__ __forceinline__ void coupling_sums(const float (&phi)[P], float (&acc)[P])
{
#pragma unroll
    for (int a = 0; a < P; ++a)
        acc[a] = 0.0f;
    // Pairs inside the lane.
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int b = a + 1; b < P; ++b) {
            const float s = sin_rev(phi[b] - phi[a]);
            acc[a] += s;
            acc[b] -= s;
        }
    }
    couple_rotations<P, 1>(phi, acc);
    // Opposite lane (rotation by 8 is its own inverse): each side adds its own.
    float other[P];
#pragma unroll
    for (int b = 0; b < P; ++b)
        other[b] = row_rotate<8>(phi[b]);
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int b = 0; b < P; ++b)
            acc[a] += sin_rev(other[b] - phi[a]);
    }
}

// Normals P*l .. P*l+P-1 of one orbit at global step k.
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
    } else {
        static_assert(P == 1, "oscillators per lane");
        const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)(l >> 2), 0u, st.key_lo, st.key_hi);
        const bool upper = (l & 2) != 0;
        float zc, zs;
        box_muller_f32(upper ? w.w2 : w.w0, upper ? w.w3 : w.w1, zc, zs);
        xi[0] = (l & 1) ? zs : zc;
    }
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

template <int P>
__device__ __forceinline__ void save(const CoupledArgs& a, int l, const float (&th)[P], float* out_row, int64_t s)
{
    constexpr int N = 16 * P;
    if (a.observable == kKuramotoR) {
        // Order parameter of Eq. (7): r = |sum_j e^{i theta_j}| / N.
        float c = 0.0f, sn = 0.0f;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const float rev = th[q] * kInvTwoPi;
            c += cos_rev(rev);
            sn += sin_rev(rev);
        }
        c = row_sum(c);
        sn = row_sum(sn);
        if (l == 0)
            out_row[s] = __builtin_sqrtf(c * c + sn * sn) * (1.0f / (float)N);
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q)
            out_row[s * N + P * l + q] = th[q];
    }
}

template <int N>
__global__ __launch_bounds__(256) void kuramoto_coupled_kernel(const CoupledArgs a)
{
    constexpr int P = N / 16;
    const int l = threadIdx.x & 15;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    // Whole rows are in or out together, so no rotation reads a finished lane.
    if (o >= a.orbits)
        return;

    const float* __restrict__ p = a.p + (a.p_per_orbit ? o * (int64_t)(2 * N + 1) : 0);
    const int q = a.observable == kKuramotoR ? 1 : N;
    float* __restrict__ out_row = a.out + o * a.nsave * q;

    float th[P], drift0[P], noise_scale[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int osc = P * l + i;
        // A phase already in range is taken as is, so that a saved state
        // passed back in continues bit-exactly.
        const float x0 = a.X0[o * N + osc];
        th[i] = __builtin_fabsf(x0) <= kPiF ? x0 : wrap_rad(x0);
        drift0[i] = p[1 + osc] * a.dt;
        noise_scale[i] = p[1 + N + osc] * a.sqdt;
    }
    const float kc = p[0] * a.coupling_dt;
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);

    save<P>(a, l, th, out_row, 0);
    uint32_t k = (uint32_t)a.step_offset;
    for (int64_t s = 1; s < a.nsave; ++s) {
        for (int64_t kk = 0; kk < a.stride; ++kk, ++k) {
            float phi[P], acc[P], xi[P];
#pragma unroll
            for (int i = 0; i < P; ++i)
                phi[i] = th[i] * kInvTwoPi;
            coupling_sums<P>(phi, acc);
            lane_normals<P>(st, k, l, xi);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                // Eq. (6): theta += omega dt + (K/N) S dt + p sqrt(dt) xi.
                const float inc = __builtin_fmaf(noise_scale[i], xi[i], __builtin_fmaf(kc, acc[i], drift0[i]));
                th[i] = wrap_rad(th[i] + inc);
            }
        }
        save<P>(a, l, th, out_row, s);
    }
}

template <int N>
hipError_t launch_n(const Request& r)
{
    CoupledArgs a;
    a.X0 = static_cast<const float*>(r.X0);
    a.p = static_cast<const float*>(r.p);
    a.out = static_cast<float*>(r.out);
    a.ids = r.orbit_ids;
    a.seeds = r.orbit_seeds;
    a.p_per_orbit = r.p_per_orbit;
    a.observable = r.observable;
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.dt = (float)r.dt;
    a.sqdt = (float)sqrt(r.dt);
    a.coupling_dt = (float)(r.dt / (double)N);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    const int64_t threads = r.orbits * 16;
    const dim3 block(256);
    const dim3 grid((unsigned)((threads + 255) / 256));
    hipLaunchKernelGGL((kuramoto_coupled_kernel<N>), grid, block, 0, r.stream, a);
    return hipGetLastError();
}

}  // namespace

bool coupled_supports(int n) { return n == 16 || n == 32 || n == 64 || n == 128; }

hipError_t launch_kuramoto_coupled_f32(const Request& r)
{
    switch (r.n) {
    case 16: return launch_n<16>(r);
    case 32: return launch_n<32>(r);
    case 64: return launch_n<64>(r);
    case 128: return launch_n<128>(r);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sode
