// kuramoto_coupled.hip - binary32 Euler-Maruyama integration of stochastic
// Kuramoto networks (Eq. 5/6 of Sec. 2.2.1) with all-to-all sine coupling,
// one orbit per 16-lane DPP row (the lane mapping, the pair evaluation and
// the padding of sizes that are not multiples of 16 are described in
// kuramoto_lanes.hpp), pairwise or through the mean-field identity.  Saves
// the state or the order parameter every `stride` steps (Sec. 2.1.4).
#include "devmath.hpp"
#include "kuramoto_lanes.hpp"
#include "launch.hpp"
#include "noise_stage.hpp"

namespace sode {
namespace {

using namespace kuramoto;

struct CoupledArgs {
    const float* __restrict__ X0;
    const float* __restrict__ p;
    float* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int n, p_per_orbit, observable;
    int64_t orbits, stride, nsave;
    float dt, sqdt, dt_over_n, inv_n;
    uint64_t seed, orbit_offset, step_offset;
    int* nonfinite;
};

// Observable of the row at save s: the state (the lane's real oscillators)
// or r (written by lane 0).
template <int P, bool PAD>
__device__ __forceinline__ void save(const CoupledArgs& a, int l, const float (&th)[P],
                                     const LaneCoefficients<P, PAD>& c, float* out_row, int64_t s)
{
    if (a.observable == kKuramotoR) {
        float r;
        if constexpr (PAD)
            r = order_parameter_padded<P>(th, c.weight, a.inv_n);
        else
            r = order_parameter<P>(th);
        if (l == 0) {
            note_nonfinite(a.nonfinite, r);
            out_row[s] = r;
        }
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int osc = P * l + q;
            if (!PAD || osc < a.n) {
                note_nonfinite(a.nonfinite, th[q]);
                out_row[s * a.n + osc] = th[q];
            }
        }
    }
}

// One orbit per 16-lane row, P oscillators per lane; PAD: the system has
// a.n < 16P oscillators and the rest of the row is padding.
template <int P, bool PAD, bool COMP, bool MF>
__global__ __launch_bounds__(256) void kuramoto_coupled_kernel(const CoupledArgs a)
{
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
    const LaneCoefficients<P, PAD> c = lane_coefficients<P, PAD>(p, l, a.dt, a.sqdt, a.dt_over_n, n);
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
                    em_step<P, COMP, MF, PAD>(th, tl, c, st, k, l, nullptr, xb[t]);
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
                em_step<P, COMP, MF, PAD>(th, tl, c, st, k, l);
            save<P, PAD>(a, l, th, c, out_row, s);
        }
    }
}

// One orbit on a 16-lane row with its normals given (the staged form of
// noise_stage.hpp): the same set-up, em_step and saves as the kernel above.
// A row past the last orbit (live = false) runs from phase 0 on orbit 0's
// coefficients and saves nothing.
template <int P, bool PAD, bool COMP, bool MF>
struct RowOrbit32 {
    static constexpr int kLanes = 16;
    static constexpr int kNormals = P;
    float th[P], tl[P];
    LaneCoefficients<P, PAD> c;
    Stream st;
    float* __restrict__ out_row;
    int l;
    bool live;

    __device__ __forceinline__ RowOrbit32(const CoupledArgs& a, int64_t o, int lane, bool is_live)
        : l(lane), live(is_live)
    {
        const int n = PAD ? a.n : 16 * P;
        const int64_t oc = live ? o : 0;
        const float* __restrict__ p = a.p + (a.p_per_orbit ? oc * (int64_t)(2 * n + 1) : 0);
        const int q = a.observable == kKuramotoR ? 1 : n;
        out_row = a.out + oc * a.nsave * q;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int osc = P * l + i;
            th[i] = live && (!PAD || osc < n) ? load_phase(a.X0[o * n + osc]) : 0.0f;
            tl[i] = 0.0f;
        }
        c = lane_coefficients<P, PAD>(p, l, a.dt, a.sqdt, a.dt_over_n, n);
        st = orbit_stream(oc, a.seed, a.orbit_offset, a.ids, a.seeds);
    }

    __device__ __forceinline__ void save(const CoupledArgs& a, int64_t s)
    {
        if (live)  // whole rows, so the row sums of r stay inside live rows
            sode::save<P, PAD>(a, l, th, c, out_row, s);
    }

    __device__ __forceinline__ void step(const float (&xi)[P])
    {
        em_step<P, COMP, MF, PAD>(th, tl, c, st, 0u, l, nullptr, xi);
    }
};

template <int P, bool PAD, bool COMP, bool MF, int NW>
__global__ __launch_bounds__(64 * (1 + NW)) void kuramoto_coupled_staged_kernel(const CoupledArgs a)
{
    __shared__ __attribute__((aligned(16))) float stage[2][kStageNormals32];
    staged_workgroup<RowOrbit32<P, PAD, COMP, MF>, float, kStageNormals32, 4, 16 * P, NW>(a, stage);
}

template <int P, bool PAD, bool COMP, bool MF>
hipError_t launch_staged(const Request& r, const CoupledArgs& a, int nw)
{
    const dim3 grid((unsigned)((r.orbits + 3) / 4));
    if (nw == 2)
        hipLaunchKernelGGL((kuramoto_coupled_staged_kernel<P, PAD, COMP, MF, 2>), grid, dim3(192), 0, r.stream, a);
    else
        hipLaunchKernelGGL((kuramoto_coupled_staged_kernel<P, PAD, COMP, MF, 1>), grid, dim3(128), 0, r.stream, a);
    return hipGetLastError();
}

template <int P, bool PAD>
hipError_t launch_p(const Request& r)
{
    CoupledArgs a;
    a.X0 = static_cast<const float*>(r.X0);
    a.p = static_cast<const float*>(r.p);
    a.out = static_cast<float*>(r.out);
    a.ids = r.orbit_ids;
    a.seeds = r.orbit_seeds;
    a.n = r.n;
    a.p_per_orbit = r.p_per_orbit;
    a.observable = r.observable;
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.dt = (float)r.dt;
    a.sqdt = (float)sqrt(r.dt);
    a.dt_over_n = (float)(r.dt / (double)r.n);
    a.inv_n = (float)(1.0 / (double)r.n);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    a.nonfinite = r.nonfinite;
    const bool mf = r.drift == 1;
    if constexpr (P == 1 || P == 2 || P == 4) {
        const int nw = staged_noise_waves(r, (r.orbits + 3) / 4);
        if (nw > 0) {
            if (r.compensated && mf)
                return launch_staged<P, PAD, true, true>(r, a, nw);
            if (r.compensated)
                return launch_staged<P, PAD, true, false>(r, a, nw);
            if (mf)
                return launch_staged<P, PAD, false, true>(r, a, nw);
            return launch_staged<P, PAD, false, false>(r, a, nw);
        }
    }
    const int64_t threads = r.orbits * 16;
    const dim3 block(256);
    const dim3 grid((unsigned)((threads + 255) / 256));
    if (r.compensated && mf)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, true, true>), grid, block, 0, r.stream, a);
    else if (r.compensated)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, true, false>), grid, block, 0, r.stream, a);
    else if (mf)
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, false, true>), grid, block, 0, r.stream, a);
    else
        hipLaunchKernelGGL((kuramoto_coupled_kernel<P, PAD, false, false>), grid, block, 0, r.stream, a);
    return hipGetLastError();
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
