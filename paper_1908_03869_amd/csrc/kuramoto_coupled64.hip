// kuramoto_coupled64.hip - binary64 Euler-Maruyama integration of stochastic
// Kuramoto networks (Eq. 5/6 of Sec. 2.2.1), 16 or 4 lanes per orbit.
//
// The binary64 counterpart of kuramoto_coupled.hip, for the precision the
// paper measured in (Sec. 2.2.1): lane l of a 16-lane DPP row owns the
// P = ceil(N/16) oscillators P*l .. P*l+P-1 (rows of N < 16P padded with
// oscillators frozen at phase 0 whose terms are cancelled, as in the binary32
// kernel); for N <= 4 a quad of lanes holds the orbit instead.  Every
// unordered pair {i, j} is evaluated once, with a binary64 sine for the
// bounded arguments these phases give (sin_phase64), and used for both
// oscillators; 64-bit values cross lanes as two 32-bit DPP moves.  The state
// is kept in radians and wrapped to [-pi, pi] every step (theta - k 2pi_hi -
// k 2pi_lo, no rounding when k = 0).  Normals come from the same Philox
// blocks and uniforms as the plain kernel's and the oracle's, through a
// Box-Muller pair that uses that the uniforms are 24-bit (box_muller_f64_u24:
// within a few ulp of the device library's functions, at about 70 % of their
// issue cost); for small ensembles other waves of the workgroup draw them.
// Compared with one orbit per lane it moves 16x (4x) more lanes through each
// step, which matters when the ensemble is too small to fill the chip (Sec.
// 2.2.1 starts at 512 orbits).
#include "devmath.hpp"
#include "launch.hpp"
#include "noise.hpp"
#include "noise_stage.hpp"
#include "phase64.hpp"

namespace sode {
namespace {

constexpr double kTwoPiHi = 6.283185307179586232;      // binary64 nearest to 2 pi
constexpr double kTwoPiLo = 2.4492935982947064e-16;    // 2 pi - kTwoPiHi
constexpr double kInvTwoPi = 0.15915494309189534561;
constexpr double kPi = 3.1415926535897931160;          // binary64 nearest to pi

// Value of `v` held by the lane R rotations away in the same 16-lane row.
template <int R>
__device__ __forceinline__ double row_rotate64(double v)
{
    static_assert(R >= 1 && R <= 15, "row rotation amount");
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x120 + R, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x120 + R, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double row_sum64(double v)
{
    v += row_rotate64<8>(v);
    v += row_rotate64<4>(v);
    v += row_rotate64<2>(v);
    v += row_rotate64<1>(v);
    return v;
}

__device__ __forceinline__ double wrap64(double x)
{
    const double k = rint(x * kInvTwoPi);
    x = fma(-k, kTwoPiHi, x);
    return fma(-k, kTwoPiLo, x);
}

__device__ __forceinline__ double load_phase64(double x) { return fabs(x) <= kPi ? x : wrap64(x); }

// Pairs between this lane and the lane K rotations away (K = 1..7, below
// LIM): this lane evaluates them and returns the negated partial sums with
// the inverse rotation.
template <int P, int K, int LIM>
__device__ __forceinline__ void couple_across64(const double (&th)[P], double (&acc)[P])
{
    if constexpr (K >= LIM)
        return;
    double other[P], back[P];
#pragma unroll
    for (int b = 0; b < P; ++b)
        other[b] = row_rotate64<16 - K>(th[b]);
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int b = 0; b < P; ++b) {
            const double s = sin_phase64(other[b] - th[a]);
            acc[a] += s;
            back[b] = a == 0 ? s : back[b] + s;
        }
    }
#pragma unroll
    for (int b = 0; b < P; ++b)
        acc[b] -= row_rotate64<K>(back[b]);
    if constexpr (K < 7)
        couple_across64<P, K + 1, LIM>(th, acc);
}

// sum_j sin(theta_j - theta_i) for the lane's P oscillators (pads included).
// LIM <= 8: only the rotations below LIM and not the opposite lane (short
// rows, see RowOrbit64).
template <int P, int LIM = 9>
__device__ __forceinline__ void coupling_sums64(const double (&th)[P], double (&acc)[P])
{
    if constexpr (P == 1) {
        acc[0] = 0.0;
    } else {
#pragma unroll
        for (int a = 0; a < P; ++a) {
#pragma unroll
            for (int b = a + 1; b < P; ++b) {
                const double s = sin_phase64(th[b] - th[a]);
                acc[a] = (a == 0 && b == 1) ? s : acc[a] + s;
                acc[b] = a == 0 ? -s : acc[b] - s;
            }
        }
    }
    couple_across64<P, 1, LIM>(th, acc);
    if constexpr (LIM <= 8)
        return;
    // Opposite lane (rotation by 8, its own inverse): pairs (own a, partner
    // b) with a < b here, returned to the partner, which covers a > b; a = b
    // by both lanes, each for its own side.
    double other[P], back[P];
#pragma unroll
    for (int b = 0; b < P; ++b)
        other[b] = row_rotate64<8>(th[b]);
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
        for (int b = a; b < P; ++b) {
            const double s = sin_phase64(other[b] - th[a]);
            acc[a] += s;
            if (b > a)
                back[b] = a == 0 ? s : back[b] + s;
        }
    }
#pragma unroll
    for (int b = 1; b < P; ++b)
        acc[b] -= row_rotate64<8>(back[b]);
}

// Binary64 normals P*l .. P*l+P-1 of one orbit at global step k: the Philox
// blocks the lane's range touches, each giving four normals in the order of
// the oracle (words 0,1 -> normals 4b, 4b+1; words 2,3 -> 4b+2, 4b+3).
template <int P>
__device__ __forceinline__ void lane_normals64(const Stream& st, uint32_t k, int l, double (&xi)[P])
{
    if constexpr (P % 4 == 0) {  // whole blocks P l / 4 .. P l / 4 + P / 4 - 1
#pragma unroll
        for (int g = 0; g < P / 4; ++g) {
            const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)((P / 4) * l + g), 0u, st.key_lo, st.key_hi);
            box_muller_f64_u24(w.w0, w.w1, xi[4 * g + 0], xi[4 * g + 1]);
            box_muller_f64_u24(w.w2, w.w3, xi[4 * g + 2], xi[4 * g + 3]);
        }
    } else {
        constexpr int NB = (P + 6) / 4;  // ceil((P + 3) / 4) blocks at most
        const int j0 = P * l;
        const int off = j0 & 3;
        double z[4 * NB];
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const Block4 w = philox_4x32_10(k, st.oid, (uint32_t)((j0 >> 2) + g), 0u, st.key_lo, st.key_hi);
            box_muller_f64_u24(w.w0, w.w1, z[4 * g + 0], z[4 * g + 1]);
            box_muller_f64_u24(w.w2, w.w3, z[4 * g + 2], z[4 * g + 3]);
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
            xi[i] = off == 0 ? z[i] : off == 1 ? z[i + 1] : off == 2 ? z[i + 2] : z[i + 3];
    }
}

// A binary64 value held by lane S of the lane's quad (two DPP quad_perm
// moves of the 32-bit halves).
template <int S>
__device__ __forceinline__ double from_quad_lane64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x55 * S, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x55 * S, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// lane_normals64<P> of the 4/P consecutive steps k .. k+4/P-1 at once
// (P = 1 or 2), xi[t] being those of step k+t: the lanes of a quad (P = 1)
// or pair (P = 2) need the normals of one Philox block per step, so each
// evaluates the block of one of the steps (and its Box-Muller pairs) and
// passes on what the others need through DPP.  The same values with 1/4 or
// 1/2 of the Philox work and 1/4 or 1/2 of the binary64 Box-Muller work.
template <int P>
__device__ __forceinline__ void lane_normals64_steps(const Stream& st, uint32_t k, int l, double (&xi)[4 / P][P])
{
    static_assert(P == 1 || P == 2, "lanes per Philox block");
    if constexpr (P == 2) {
        const bool odd = (l & 1) != 0;
        const Block4 w = philox_4x32_10(k + (odd ? 1u : 0u), st.oid, (uint32_t)(l >> 1), 0u, st.key_lo, st.key_hi);
        const uint32_t own0 = odd ? w.w2 : w.w0, own1 = odd ? w.w3 : w.w1;
        const uint32_t got0 = from_pair_lane(odd ? w.w0 : w.w2);
        const uint32_t got1 = from_pair_lane(odd ? w.w1 : w.w3);
        box_muller_f64_u24(odd ? got0 : own0, odd ? got1 : own1, xi[0][0], xi[0][1]);
        box_muller_f64_u24(odd ? own0 : got0, odd ? own1 : got1, xi[1][0], xi[1][1]);
    } else {
        const int qi = l & 3;
        const Block4 w = philox_4x32_10(k + (uint32_t)qi, st.oid, (uint32_t)(l >> 2), 0u, st.key_lo, st.key_hi);
        double z0, z1, z2, z3;
        box_muller_f64_u24(w.w0, w.w1, z0, z1);
        box_muller_f64_u24(w.w2, w.w3, z2, z3);
        auto mine = [qi](double c0, double c1, double c2, double c3) {
            return (qi & 2) ? ((qi & 1) ? c3 : c2) : ((qi & 1) ? c1 : c0);
        };
        xi[0][0] = mine(from_quad_lane64<0>(z0), from_quad_lane64<0>(z1), from_quad_lane64<0>(z2),
                        from_quad_lane64<0>(z3));
        xi[1][0] = mine(from_quad_lane64<1>(z0), from_quad_lane64<1>(z1), from_quad_lane64<1>(z2),
                        from_quad_lane64<1>(z3));
        xi[2][0] = mine(from_quad_lane64<2>(z0), from_quad_lane64<2>(z1), from_quad_lane64<2>(z2),
                        from_quad_lane64<2>(z3));
        xi[3][0] = mine(from_quad_lane64<3>(z0), from_quad_lane64<3>(z1), from_quad_lane64<3>(z2),
                        from_quad_lane64<3>(z3));
    }
}

struct Coupled64Args {
    const double* __restrict__ X0;
    const double* __restrict__ p;
    double* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int n, p_per_orbit, observable;
    int64_t orbits, stride, nsave;
    double dt, sqdt;
    uint64_t seed, orbit_offset, step_offset;
    int* nonfinite;
};

// r of Eq. (7) over the n real oscillators of the row.
template <int P>
__device__ __forceinline__ double order_parameter64(const double (&th)[P], const double (&w)[P], int n)
{
    double c = 0.0, s = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        c += cos(th[q]) * w[q];
        s += sin(th[q]) * w[q];
    }
    const double C = row_sum64(c), S = row_sum64(s);
    return sqrt(C * C + S * S) / (double)n;
}

// A binary64 value held by another lane of the same quad, selected by the
// DPP quad_perm control CTRL (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double quad_perm64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// quad_perm selections (lane i of a quad takes lane sel[i]):
constexpr int kQuadNext = 0x39;  // [1, 2, 3, 0]: lane (l + 1) mod 4
constexpr int kQuadPrev = 0x93;  // [3, 0, 1, 2]: lane (l - 1) mod 4
constexpr int kQuadOpp = 0x4E;   // [2, 3, 0, 1]: lane (l + 2) mod 4

__device__ __forceinline__ double quad_sum64(double v)
{
    v += quad_perm64<kQuadOpp>(v);
    return v + quad_perm64<kQuadNext>(v);
}

// One orbit on a 16-lane row (Sec. 2.2.1, Eq. 5/6): lane l's P oscillators,
// their per-oscillator constants (omega dt, p sqrt(dt), K dt / N, weight 0
// for pads), the save of the state or of r, and one Euler-Maruyama step
// with given normals.  A row past the last orbit (live = false) runs on
// zeros and saves nothing; it reads no input.  LIM <= 8: a short row of
// a.n = LIM oscillators, one per lane: lanes LIM .. 15 are pads, the
// rotations by LIM .. 7 and by 8 pair real lanes with pads only and are left
// out, and every real lane meets LIM - 1 pads (i through its own rotations,
// LIM - 1 - i through the pads' returns) instead of 16 - LIM.
template <int P, bool PAD, bool MF, int LIM = 9>
struct RowOrbit64 {
    static_assert(LIM > 8 || (P == 1 && PAD && !MF), "short rows: one padded oscillator per lane, pairwise");
    static constexpr int kLanes = 16;  // lanes per orbit
    static constexpr int kNormals = P; // normals per lane and step
    double th[P], drift0[P], noise[P], kc[P], w[P];
    double pads;
    double* __restrict__ out_row;
    int l, n;
    bool live;

    __device__ __forceinline__ RowOrbit64(const Coupled64Args& a, int64_t o, int lane, bool is_live)
        : l(lane), n(PAD ? a.n : 16 * P), live(is_live)
    {
        const int64_t oc = live ? o : 0;
        const double* __restrict__ p = a.p + (a.p_per_orbit ? oc * (int64_t)(2 * n + 1) : 0);
        const int q = a.observable == kKuramotoR ? 1 : n;
        out_row = a.out + oc * a.nsave * q;
        const double kcv = live ? p[0] * (a.dt / (double)n) : 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int osc = P * l + i;
            const bool real = live && (!PAD || osc < n);
            th[i] = real ? load_phase64(a.X0[o * n + osc]) : 0.0;
            drift0[i] = real ? p[1 + osc] * a.dt : 0.0;
            noise[i] = real ? p[1 + n + osc] * a.sqdt : 0.0;
            kc[i] = real ? kcv : 0.0;
            w[i] = real ? 1.0 : 0.0;
        }
        pads = (double)(LIM <= 8 ? n - 1 : 16 * P - n);
    }

    __device__ __forceinline__ void save(const Coupled64Args& a, int64_t s)
    {
        if (a.observable == kKuramotoR) {
            const double r = order_parameter64<P>(th, w, n);
            if (live && l == 0) {
                note_nonfinite(a.nonfinite, r);
                out_row[s] = r;
            }
        } else {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int osc = P * l + i;
                if (live && (!PAD || osc < n)) {
                    note_nonfinite(a.nonfinite, th[i]);
                    out_row[s * n + osc] = th[i];
                }
            }
        }
    }

    __device__ __forceinline__ void step(const double (&xi)[P])
    {
        double acc[P];
        if constexpr (MF) {
            // sum_j sin(theta_j - theta_i) = cos(theta_i) S - sin(theta_i) C.
            double cs[P], sn[P], c = 0.0, sv = 0.0;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                sincos(th[i], &sn[i], &cs[i]);
                c += cs[i] * w[i];
                sv += sn[i] * w[i];
            }
            const double C = row_sum64(c), S = row_sum64(sv);
#pragma unroll
            for (int i = 0; i < P; ++i)
                acc[i] = cs[i] * S - sn[i] * C;
        } else {
            coupling_sums64<P, LIM>(th, acc);
            if constexpr (PAD) {
#pragma unroll
                for (int i = 0; i < P; ++i)
                    acc[i] = fma(pads, sin_phase64(th[i]), acc[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
            th[i] = wrap64(th[i] + (fma(kc[i], acc[i], drift0[i]) + noise[i] * xi[i]));
    }
};

// n <= 4: one orbit per quad of lanes, one oscillator per lane (lanes
// l >= n hold pads at phase 0, cancelled as in the row form).  Every
// unordered pair is evaluated once: the pairs (l, l + 1 mod 4) by lane l,
// which returns the negated sine to lane l + 1, and the pairs (l, l + 2
// mod 4) by both of their lanes.  Two binary64 sines per lane and step
// instead of the 16-lane row's eight (and 16 lanes per orbit instead of 4).
template <bool PAD, bool MF>
struct QuadOrbit64 {
    static constexpr int kLanes = 4;
    static constexpr int kNormals = 1;
    double th, drift0, noise, kc, w, pads;
    double* __restrict__ out_row;
    int l, n;
    bool live, real;

    __device__ __forceinline__ QuadOrbit64(const Coupled64Args& a, int64_t o, int lane, bool is_live)
        : l(lane), n(PAD ? a.n : 4), live(is_live), real(is_live && (!PAD || lane < n))
    {
        const int64_t oc = live ? o : 0;
        const double* __restrict__ p = a.p + (a.p_per_orbit ? oc * (int64_t)(2 * n + 1) : 0);
        const int q = a.observable == kKuramotoR ? 1 : n;
        out_row = a.out + oc * a.nsave * q;
        th = real ? load_phase64(a.X0[o * n + l]) : 0.0;
        drift0 = real ? p[1 + l] * a.dt : 0.0;
        noise = real ? p[1 + n + l] * a.sqdt : 0.0;
        kc = real ? p[0] * (a.dt / (double)n) : 0.0;
        w = real ? 1.0 : 0.0;
        pads = (double)(4 - n);
    }

    __device__ __forceinline__ void save(const Coupled64Args& a, int64_t s)
    {
        if (a.observable == kKuramotoR) {
            const double C = quad_sum64(cos(th) * w), S = quad_sum64(sin(th) * w);
            const double r = sqrt(C * C + S * S) / (double)n;
            if (live && l == 0) {
                note_nonfinite(a.nonfinite, r);
                out_row[s] = r;
            }
        } else if (real) {
            note_nonfinite(a.nonfinite, th);
            out_row[s * n + l] = th;
        }
    }

    __device__ __forceinline__ void step(const double (&xi)[1])
    {
        double acc;
        if constexpr (MF) {
            double sn, cs;
            sincos(th, &sn, &cs);
            const double C = quad_sum64(cs * w), S = quad_sum64(sn * w);
            acc = cs * S - sn * C;
        } else {
            const double s1 = sin_phase64(quad_perm64<kQuadNext>(th) - th);
            acc = s1 - quad_perm64<kQuadPrev>(s1);
            acc += sin_phase64(quad_perm64<kQuadOpp>(th) - th);
            if constexpr (PAD)
                acc = fma(pads, sin_phase64(th), acc);
        }
        th = wrap64(th + (fma(kc, acc, drift0) + noise * xi[0]));
    }
};

// The row and quad forms with each lane drawing its own normals (several
// steps at a time where lanes share a Philox block), one orbit per row or
// quad, 256-thread blocks.  Whole rows and quads are in or out together, so
// no lane permutation reads a finished lane.
template <int P, bool PAD, bool MF, int LIM = 9>
__global__ __launch_bounds__(256) void kuramoto_coupled64_kernel(const Coupled64Args a)
{
    const int l = threadIdx.x & 15;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (o >= a.orbits)
        return;
    RowOrbit64<P, PAD, MF, LIM> f(a, o, l, true);
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);
    f.save(a, 0);
    uint32_t k = (uint32_t)a.step_offset;
    if constexpr (P <= 2) {
        // Normals of B = 4/P steps at a time (lane_normals64_steps).
        constexpr int B = 4 / P;
        const int64_t nsteps = (a.nsave - 1) * a.stride;
        int64_t s = 1, to_save = a.stride;
        for (int64_t j = 0; j < nsteps; j += B) {
            double xb[B][P];
            lane_normals64_steps<P>(st, k, l, xb);
#pragma unroll
            for (int t = 0; t < B; ++t) {
                if (t == 0 || j + t < nsteps) {
                    f.step(xb[t]);
                    ++k;
                    if (__builtin_expect(--to_save == 0, 0)) {
                        f.save(a, s);
                        ++s;
                        to_save = a.stride;
                    }
                }
            }
        }
    } else {
        for (int64_t s = 1; s < a.nsave; ++s) {
            for (int64_t kk = 0; kk < a.stride; ++kk, ++k) {
                double xi[P];
                lane_normals64<P>(st, k, l, xi);
                f.step(xi);
            }
            f.save(a, s);
        }
    }
}

template <bool PAD, bool MF>
__global__ __launch_bounds__(256) void kuramoto_quad64_kernel(const Coupled64Args a)
{
    const int l = threadIdx.x & 3;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    if (o >= a.orbits)
        return;
    QuadOrbit64<PAD, MF> f(a, o, l, true);
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);
    f.save(a, 0);
    uint32_t k = (uint32_t)a.step_offset;
    const int64_t nsteps = (a.nsave - 1) * a.stride;
    int64_t s = 1, to_save = a.stride;
    for (int64_t j = 0; j < nsteps; j += 4) {
        double xb[4][1];
        lane_normals64_steps<1>(st, k, l, xb);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t == 0 || j + t < nsteps) {
                f.step(xb[t]);
                ++k;
                if (__builtin_expect(--to_save == 0, 0)) {
                    f.save(a, s);
                    ++s;
                    to_save = a.stride;
                }
            }
        }
    }
}

// The same forms with their normals drawn by other waves of the workgroup
// (noise_stage.hpp): one integrating wave of G orbits (16 quads or 4 rows).
template <class Orbit, int G, int NPO, int NW>
__global__ __launch_bounds__(64 * (1 + NW)) void coupled64_staged_kernel(const Coupled64Args a)
{
    __shared__ __attribute__((aligned(16))) double stage[2][kStageNormals64];
    staged_workgroup<Orbit, double, kStageNormals64, G, NPO, NW>(a, stage);
}

template <class Orbit, int G, int NPO>
hipError_t launch_staged64(const Request& r, const Coupled64Args& a, int nw)
{
    const dim3 grid((unsigned)((r.orbits + G - 1) / G));
    if (nw == 2)
        hipLaunchKernelGGL((coupled64_staged_kernel<Orbit, G, NPO, 2>), grid, dim3(192), 0, r.stream, a);
    else
        hipLaunchKernelGGL((coupled64_staged_kernel<Orbit, G, NPO, 1>), grid, dim3(128), 0, r.stream, a);
    return hipGetLastError();
}

template <bool PAD>
hipError_t launch_quad64(const Request& r, const Coupled64Args& a)
{
    const int nw = staged_noise_waves(r, (r.orbits + 15) / 16);
    if (nw > 0)
        return r.drift == 1 ? launch_staged64<QuadOrbit64<PAD, true>, 16, 4>(r, a, nw)
                            : launch_staged64<QuadOrbit64<PAD, false>, 16, 4>(r, a, nw);
    const dim3 grid((unsigned)((r.orbits * 4 + 255) / 256));
    if (r.drift == 1)
        hipLaunchKernelGGL((kuramoto_quad64_kernel<PAD, true>), grid, dim3(256), 0, r.stream, a);
    else
        hipLaunchKernelGGL((kuramoto_quad64_kernel<PAD, false>), grid, dim3(256), 0, r.stream, a);
    return hipGetLastError();
}

// Pairwise rows of 5 <= n <= 8 oscillators, one per lane, staged or not:
// the coupling sums leave out the rotations that reach pads only (LIM = n).
template <int LIM>
hipError_t launch_short_row64(const Request& r, const Coupled64Args& a)
{
    const int nw = staged_noise_waves(r, (r.orbits + 3) / 4);
    if (nw > 0)
        return launch_staged64<RowOrbit64<1, true, false, LIM>, 4, 16>(r, a, nw);
    const dim3 grid((unsigned)((r.orbits * 16 + 255) / 256));
    hipLaunchKernelGGL((kuramoto_coupled64_kernel<1, true, false, LIM>), grid, dim3(256), 0, r.stream, a);
    return hipGetLastError();
}

template <int P, bool PAD>
hipError_t launch_p64(const Request& r)
{
    Coupled64Args a;
    a.X0 = static_cast<const double*>(r.X0);
    a.p = static_cast<const double*>(r.p);
    a.out = static_cast<double*>(r.out);
    a.ids = r.orbit_ids;
    a.seeds = r.orbit_seeds;
    a.n = r.n;
    a.p_per_orbit = r.p_per_orbit;
    a.observable = r.observable;
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.dt = r.dt;
    a.sqdt = sqrt(r.dt);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    a.nonfinite = r.nonfinite;
    if (P == 1 && r.n <= 4)  // four lanes per orbit
        return r.n == 4 ? launch_quad64<false>(r, a) : launch_quad64<true>(r, a);
    if constexpr (P == 1 && PAD) {
        if (r.drift != 1) {
            switch (r.n) {
            case 5: return launch_short_row64<5>(r, a);
            case 6: return launch_short_row64<6>(r, a);
            case 7: return launch_short_row64<7>(r, a);
            case 8: return launch_short_row64<8>(r, a);
            default: break;
            }
        }
    }
    if constexpr (P == 1 || P == 2 || P == 4) {
        const int nw = staged_noise_waves(r, (r.orbits + 3) / 4);
        if (nw > 0)
            return r.drift == 1 ? launch_staged64<RowOrbit64<P, PAD, true>, 4, 16 * P>(r, a, nw)
                                : launch_staged64<RowOrbit64<P, PAD, false>, 4, 16 * P>(r, a, nw);
    }
    const dim3 grid((unsigned)((r.orbits * 16 + 255) / 256));
    if (r.drift == 1)
        hipLaunchKernelGGL((kuramoto_coupled64_kernel<P, PAD, true>), grid, dim3(256), 0, r.stream, a);
    else
        hipLaunchKernelGGL((kuramoto_coupled64_kernel<P, PAD, false>), grid, dim3(256), 0, r.stream, a);
    return hipGetLastError();
}

template <int P>
hipError_t launch_padded_or_not64(const Request& r)
{
    if (r.n == 16 * P)
        return launch_p64<P, false>(r);
    return launch_p64<P, true>(r);
}

}  // namespace

hipError_t launch_kuramoto_coupled_f64(const Request& r)
{
    switch ((r.n + 15) / 16) {
    case 1: return launch_padded_or_not64<1>(r);
    case 2: return launch_padded_or_not64<2>(r);
    case 3: return launch_p64<3, true>(r);
    case 4: return launch_padded_or_not64<4>(r);
    default: return hipErrorInvalidValue;
    }
}

bool coupled64_supports(int n) { return n >= 1 && n <= 64; }

}  // namespace sode
