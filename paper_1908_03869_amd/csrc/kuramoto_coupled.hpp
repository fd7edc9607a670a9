// kuramoto_coupled.hpp - what the binary32 coupled Kuramoto kernels share:
// the kernel argument block, the save of the state or the order parameter
// every `stride` steps (Sec. 2.1.4) and its host-side fill.  The unstaged
// kernels (kuramoto_coupled.hip) and the staged ones (their normals drawn by
// other waves of the workgroup, kuramoto_coupled_staged.hip) live in
// separate translation units so that each is compiled on its own.
#pragma once

#include <cmath>

#include "devmath.hpp"
#include "kuramoto_lanes.hpp"
#include "launch.hpp"

namespace sode {
namespace coupled32 {

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

inline CoupledArgs coupled_args(const Request& r)
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
    a.sqdt = (float)std::sqrt(r.dt);
    a.dt_over_n = (float)(r.dt / (double)r.n);
    a.inv_n = (float)(1.0 / (double)r.n);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    a.nonfinite = r.nonfinite;
    return a;
}

// The staged form for rows of P = 1, 2 or 4 oscillators per lane, nw = 1 or
// 2 noise waves per workgroup of four rows (kuramoto_coupled_staged.hip).
hipError_t launch_staged_f32(const Request& r, const CoupledArgs& a, int nw);

}  // namespace coupled32
}  // namespace sode
