// kuramoto_coupled.hip - binary32 Euler-Maruyama integration of stochastic
// Kuramoto networks (Eq. 5/6 of Sec. 2.2.1) with all-to-all sine coupling,
// one orbit per 16-lane DPP row (the lane mapping and the pair evaluation
// are described in kuramoto_lanes.hpp), pairwise or through the mean-field
// identity.  Saves the state or the order parameter every `stride` steps
// (Sec. 2.1.4).
#include "kuramoto_lanes.hpp"
#include "launch.hpp"

namespace sode {
namespace {

using namespace kuramoto;

struct CoupledArgs {
    const float* __restrict__ X0;
    const float* __restrict__ p;
    float* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int p_per_orbit, observable, compensated, drift;
    int64_t orbits, stride, nsave;
    float dt, sqdt, dt_over_n;
    uint64_t seed, orbit_offset, step_offset;
};

template <int P>
__device__ __forceinline__ void save(const CoupledArgs& a, int l, const float (&th)[P], float* out_row, int64_t s)
{
    constexpr int N = 16 * P;
    if (a.observable == kKuramotoR) {
        const float r = order_parameter<P>(th);
        if (l == 0)
            out_row[s] = r;
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q)
            out_row[s * N + P * l + q] = th[q];
    }
}

template <int N, bool COMP, bool MF>
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

    float th[P], tl[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        th[i] = load_phase(a.X0[o * N + P * l + i]);
        tl[i] = 0.0f;
    }
    const LaneCoefficients<P> c = lane_coefficients<P>(p, l, a.dt, a.sqdt, a.dt_over_n);
    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);

    save<P>(a, l, th, out_row, 0);
    uint32_t k = (uint32_t)a.step_offset;
    for (int64_t s = 1; s < a.nsave; ++s) {
        for (int64_t kk = 0; kk < a.stride; ++kk, ++k)
            em_step<P, COMP, MF>(th, tl, c, st, k, l);
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
    a.compensated = r.compensated;
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.dt = (float)r.dt;
    a.sqdt = (float)sqrt(r.dt);
    a.dt_over_n = (float)(r.dt / (double)N);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    const int64_t threads = r.orbits * 16;
    const dim3 block(256);
    const dim3 grid((unsigned)((threads + 255) / 256));
    if (r.drift == 1) {
        if (r.compensated)
            hipLaunchKernelGGL((kuramoto_coupled_kernel<N, true, true>), grid, block, 0, r.stream, a);
        else
            hipLaunchKernelGGL((kuramoto_coupled_kernel<N, false, true>), grid, block, 0, r.stream, a);
    } else {
        if (r.compensated)
            hipLaunchKernelGGL((kuramoto_coupled_kernel<N, true, false>), grid, block, 0, r.stream, a);
        else
            hipLaunchKernelGGL((kuramoto_coupled_kernel<N, false, false>), grid, block, 0, r.stream, a);
    }
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
