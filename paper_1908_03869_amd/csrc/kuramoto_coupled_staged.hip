// kuramoto_coupled_staged.hip - the binary32 coupled Kuramoto rows of
// kuramoto_coupled.hip with their normals drawn ahead by one or two other
// waves of the workgroup into LDS (noise_stage.hpp), for ensembles too small
// to fill the chip: the same set-up, Euler-Maruyama step (Eq. 5/6 of
// Sec. 2.2.1) and saves, so the results are bitwise those of the unstaged
// kernels.
#include "kuramoto_coupled.hpp"
#include "noise_stage.hpp"

namespace sode {
namespace coupled32 {
namespace {

// One orbit on a 16-lane row with its normals given (the staged form of
// noise_stage.hpp): the same set-up, em_step and saves as
// kuramoto_coupled_kernel.
// A row past the last orbit (live = false) runs from phase 0 on orbit 0's
// coefficients and saves nothing.
template <int P, bool PAD, bool COMP, bool MF, int LIM = 9>
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
        c = lane_coefficients<P, PAD>(p, l, a.dt, a.sqdt, a.dt_over_n, n, LIM <= 8);
        st = orbit_stream(oc, a.seed, a.orbit_offset, a.ids, a.seeds);
    }

    __device__ __forceinline__ void save(const CoupledArgs& a, int64_t s)
    {
        if (live)  // whole rows, so the row sums of r stay inside live rows
            coupled32::save<P, PAD>(a, l, th, c, out_row, s);
    }

    __device__ __forceinline__ void step(const float (&xi)[P])
    {
        em_step<P, COMP, MF, PAD, false, LIM>(th, tl, c, st, 0u, l, nullptr, xi);
    }
};

template <int P, bool PAD, bool COMP, bool MF, int NW, int LIM = 9>
__global__ __launch_bounds__(64 * (1 + NW)) void kuramoto_coupled_staged_kernel(const CoupledArgs a)
{
    __shared__ __attribute__((aligned(16))) float stage[2][kStageNormals32];
    staged_workgroup<RowOrbit32<P, PAD, COMP, MF, LIM>, float, kStageNormals32, 4, 16 * P, NW>(a, stage);
}

template <int P, bool PAD, bool COMP, bool MF, int LIM = 9>
hipError_t launch_staged(const Request& r, const CoupledArgs& a, int nw)
{
    const dim3 grid((unsigned)((r.orbits + 3) / 4));
    if (nw == 2)
        hipLaunchKernelGGL((kuramoto_coupled_staged_kernel<P, PAD, COMP, MF, 2, LIM>), grid, dim3(192), 0, r.stream,
                           a);
    else
        hipLaunchKernelGGL((kuramoto_coupled_staged_kernel<P, PAD, COMP, MF, 1, LIM>), grid, dim3(128), 0, r.stream,
                           a);
    return hipGetLastError();
}

// Pairwise rows of n <= 8 oscillators, one per lane, as in the unstaged
// kernel: the coupling sums leave out the rotations that reach pads only.
template <int LIM>
hipError_t launch_short_row(const Request& r, const CoupledArgs& a, int nw)
{
    if (r.compensated)
        return launch_staged<1, true, true, false, LIM>(r, a, nw);
    return launch_staged<1, true, false, false, LIM>(r, a, nw);
}

template <int P, bool PAD>
hipError_t launch_p(const Request& r, const CoupledArgs& a, int nw)
{
    const bool mf = r.drift == 1;
    if constexpr (P == 1 && PAD) {
        if (!mf) {
            switch (r.n) {
            case 1: return launch_short_row<1>(r, a, nw);
            case 2: return launch_short_row<2>(r, a, nw);
            case 3: return launch_short_row<3>(r, a, nw);
            case 4: return launch_short_row<4>(r, a, nw);
            case 5: return launch_short_row<5>(r, a, nw);
            case 6: return launch_short_row<6>(r, a, nw);
            case 7: return launch_short_row<7>(r, a, nw);
            case 8: return launch_short_row<8>(r, a, nw);
            default: break;
            }
        }
    }
    if (r.compensated && mf)
        return launch_staged<P, PAD, true, true>(r, a, nw);
    if (r.compensated)
        return launch_staged<P, PAD, true, false>(r, a, nw);
    if (mf)
        return launch_staged<P, PAD, false, true>(r, a, nw);
    return launch_staged<P, PAD, false, false>(r, a, nw);
}

template <int P>
hipError_t launch_padded_or_not(const Request& r, const CoupledArgs& a, int nw)
{
    if (r.n == 16 * P)
        return launch_p<P, false>(r, a, nw);
    return launch_p<P, true>(r, a, nw);
}

}  // namespace

hipError_t launch_staged_f32(const Request& r, const CoupledArgs& a, int nw)
{
    if (nw != 1 && nw != 2)
        return hipErrorInvalidValue;
    switch ((r.n + 15) / 16) {
    case 1: return launch_padded_or_not<1>(r, a, nw);
    case 2: return launch_padded_or_not<2>(r, a, nw);
    case 4: return launch_padded_or_not<4>(r, a, nw);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace coupled32
}  // namespace sode
