// kuramoto_coupled.hip - binary32 Euler-Maruyama integration of stochastic
// Kuramoto networks (Eq. 5/6 of Sec. 2.2.1) with all-to-all sine coupling,
// one orbit per 16-lane DPP row (the lane mapping, the pair evaluation and
// the padding of sizes that are not multiples of 16 are described in
// kuramoto_lanes.hpp), pairwise or through the mean-field identity.  Saves
// the state or the order parameter every `stride` steps (Sec. 2.1.4).
#include "kuramoto_coupled.hpp"
#include "noise_stage.hpp"

namespace sode {
namespace {

using namespace coupled32;

// One orbit per 16-lane row, P oscillators per lane; PAD: the system has
// a.n < 16P oscillators and the rest of the row is padding.  LDS: partner
// phases through LDS (kLdsPartnerPhases rows only), else by DPP.  LIM <= 8:
// a short row of a.n = LIM oscillators, one per lane (lane_coefficients).
template <int P, bool PAD, bool COMP, bool MF, bool LDS, int LIM = 9>
__global__ __launch_bounds__(256) void kuramoto_coupled_kernel(const CoupledArgs a)
{
    static_assert(LIM > 8 || (P == 1 && PAD && !MF), "short rows: one padded oscillator per lane, pairwise");
    static_assert(!LDS || kLdsPartnerPhases<P, MF>, "LDS partner phases for rows of 2, 4 or 8, pairwise");
    __shared__ __attribute__((aligned(16))) float lds_phase[LDS ? 256 * P : 1];
    float* const row = LDS ? lds_phase + (threadIdx.x & ~15u) * P : nullptr;
    const int l = threadIdx.x & 15;
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    // Whole rows are in or out together, so no rotation reads a finished lane.
    if (o >= a.orbits)
        return;
    const int n = PAD ? a.n : 16 * P;

    const float* __restrict__ p = a.p + (a.p_per_orbit ? o * (int64_t)(2 * n + 1) : 0);
    const int q = a.observable == kKuramotoR ? 1 : n;
    float* __restrict__ out_row = a.out + o * a.nsave * q;

    float th[P], tl[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int osc = P * l + i;
        th[i] = (!PAD || osc < n) ? load_phase(a.X0[o * n + osc]) : 0.0f;
        tl[i] = 0.0f;
    }
    const LaneCoefficients<P, PAD> c = lane_coefficients<P, PAD>(p, l, a.dt, a.sqdt, a.dt_over_n, n, LIM <= 8);
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);

    save<P, PAD>(a, l, th, c, out_row, 0);
    uint32_t k = (uint32_t)a.step_offset;
    if constexpr (P <= 2) {
        // One Philox block per quad (P = 1) or pair (P = 2) of lanes and
        // step: the normals of B = 4/P steps at a time (lane_normals_steps).
        constexpr int B = 4 / P;
        const int64_t nsteps = (a.nsave - 1) * a.stride;
        int64_t s = 1, to_save = a.stride;
        for (int64_t j = 0; j < nsteps; j += B) {
            float xb[B][P];
            lane_normals_steps<P>(st, k, l, xb);
#pragma unroll
            for (int t = 0; t < B; ++t) {
                if (t == 0 || j + t < nsteps) {
                    em_step<P, COMP, MF, PAD, LDS, LIM>(th, tl, c, st, k, l, nullptr, xb[t], row);
                    ++k;
                    if (--to_save == 0) {
                        save<P, PAD>(a, l, th, c, out_row, s);
                        ++s;
                        to_save = a.stride;
                    }
                }
            }
        }
    } else {
        for (int64_t s = 1; s < a.nsave; ++s) {
            for (int64_t kk = 0; kk < a.stride; ++kk, ++k)
                em_step<P, COMP, MF, PAD, LDS, LIM>(th, tl, c, st, k, l, nullptr, nullptr, row);
            save<P, PAD>(a, l, th, c, out_row, s);
        }
    }
}

// Pairwise rows of n <= 8 oscillators, one per lane: the coupling sums
// leave out the rotations that reach pads only (LIM = n).
template <int LIM>
hipError_t launch_short_row(const Request& r, const CoupledArgs& a, dim3 grid, dim3 block)
{
    if (r.compensated)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<1, true, true, false, false, LIM>), grid, block, 0, r.stream, a);
    else
        hipLaunchKernelGGL((kuramoto_coupled_kernel<1, true, false, false, false, LIM>), grid, block, 0, r.stream, a);
    return hipGetLastError();
}

template <int P, bool PAD, bool LDS>
hipError_t launch_rows(const Request& r, const CoupledArgs& a)
{
    const bool mf = r.drift == 1;
    const int64_t threads = r.orbits * 16;
    const dim3 block(256);
    const dim3 grid((unsigned)((threads + 255) / 256));
    if constexpr (P == 1 && PAD) {
        if (!mf) {
            switch (r.n) {
            case 1: return launch_short_row<1>(r, a, grid, block);
            case 2: return launch_short_row<2>(r, a, grid, block);
            case 3: return launch_short_row<3>(r, a, grid, block);
            case 4: return launch_short_row<4>(r, a, grid, block);
            case 5: return launch_short_row<5>(r, a, grid, block);
            case 6: return launch_short_row<6>(r, a, grid, block);
            case 7: return launch_short_row<7>(r, a, grid, block);
            case 8: return launch_short_row<8>(r, a, grid, block);
            default: break;
            }
        }
    }
    if (r.compensated && mf)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, true, true, false>), grid, block, 0, r.stream, a);
    else if (r.compensated)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, true, false, LDS>), grid, block, 0, r.stream, a);
    else if (mf)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, false, true, false>), grid, block, 0, r.stream, a);
    else
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, false, false, LDS>), grid, block, 0, r.stream, a);
    return hipGetLastError();
}

template <int P, bool PAD>
hipError_t launch_p(const Request& r)
{
    const CoupledArgs a = coupled_args(r);
    if constexpr (P == 1 || P == 2 || P == 4) {
        // Small ensembles: the staged rows of kuramoto_coupled_staged.hip.
        const int nw = staged_noise_waves(r, (r.orbits + 3) / 4);
        if (nw > 0)
            return launch_staged_f32(r, a, nw);
    }
    if constexpr (kLdsPartnerPhases<P, false>) {
        // Partner phases through LDS once the SIMDs hold enough row waves to
        // hide the loads' latency: from 8 waves per SIMD with 4 oscillators
        // per lane, from 2 with 2 or 8; with fewer the DPP form is faster.
        // Either form gives the same results.
        const int64_t waves_per_simd = r.orbits / (16 * (int64_t)device_compute_units());
        if (r.drift != 1 && waves_per_simd >= (P == 4 ? 8 : 2))
            return launch_rows<P, PAD, true>(r, a);
    }
    return launch_rows<P, PAD, false>(r, a);
}

template <int P>
hipError_t launch_padded_or_not(const Request& r)
{
    if (r.n == 16 * P)
        return launch_p<P, false>(r);
    return launch_p<P, true>(r);
}

}  // namespace

bool coupled_supports(int n) { return n >= 1 && n <= 128; }

hipError_t launch_kuramoto_coupled_f32(const Request& r)
{
    switch ((r.n + 15) / 16) {
    case 1: return launch_padded_or_not<1>(r);
    case 2: return launch_padded_or_not<2>(r);
    case 3: return launch_p<3, true>(r);
    case 4: return launch_padded_or_not<4>(r);
    case 5: return launch_p<5, true>(r);
    case 6: return launch_p<6, true>(r);
    case 7: return launch_p<7, true>(r);
    case 8: return launch_padded_or_not<8>(r);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sode
