// plain_fixed.hip - the explicit steppers of the one-orbit-per-lane kernel
// (Euler-Maruyama, Milstein, RK4) with the state dimension as a compile-time
// constant, for the small Ornstein-Uhlenbeck and geometric Brownian motion
// systems (n = 2, 3, 4) and FitzHugh-Nagumo chains (n = 2, 4, 6, 8).  The
// runtime-n kernel of plain.hip keeps the state, drift and noise vectors in
// private memory, sized for its largest n; with n known they live in
// registers.  The arithmetic, and so the result, is the same bit for bit.
#include "launch.hpp"
#include "models.hpp"
#include "plain_kernel.hpp"

namespace sode {
namespace {

template <class Model, typename R, int NC, int METH>
__global__ __launch_bounds__(64) void plain_fixed_kernel(const PlainArgs<R> a)
{
    plain_body<Model, R, NC, METH, NC>(a);
}

template <class Model, typename R, int NC>
hipError_t launch_n(const Request& r)
{
    const PlainArgs<R> a = plain_args<R>(r);
    const dim3 grid((unsigned)((r.orbits + 63) / 64));
    if (r.method == kRK4)
        hipLaunchKernelGGL((plain_fixed_kernel<Model, R, NC, kRK4>), grid, dim3(64), 0, r.stream, a);
    else if (r.method == kMilstein && Model::kStateNoise)
        hipLaunchKernelGGL((plain_fixed_kernel<Model, R, NC, (Model::kStateNoise ? kMilstein : kEM)>),
                           grid, dim3(64), 0, r.stream, a);
    else  // EM; and Milstein with state-independent noise, where the correction is zero
        hipLaunchKernelGGL((plain_fixed_kernel<Model, R, NC, kEM>), grid, dim3(64), 0, r.stream, a);
    return hipGetLastError();
}

template <class Model, typename R>
bool launch_small(const Request& r, hipError_t* e)
{
    switch (r.n) {
    case 2: *e = launch_n<Model, R, 2>(r); return true;
    case 3: *e = launch_n<Model, R, 3>(r); return true;
    case 4: *e = launch_n<Model, R, 4>(r); return true;
    default: return false;
    }
}

template <typename R>
bool launch_fixed(const Request& r, hipError_t* e)
{
    switch (r.model) {
    case kOU: return launch_small<OrnsteinUhlenbeck, R>(r, e);
    case kGBM: return launch_small<GeometricBM, R>(r, e);
    case kFHN:
        switch (r.n) {
        case 2: *e = launch_n<FhnChain, R, 2>(r); return true;
        case 4: *e = launch_n<FhnChain, R, 4>(r); return true;
        case 6: *e = launch_n<FhnChain, R, 6>(r); return true;
        case 8: *e = launch_n<FhnChain, R, 8>(r); return true;
        default: return false;
        }
    default: return false;
    }
}

}  // namespace

bool launch_plain_fixed_f64(const Request& r, hipError_t* e) { return launch_fixed<double>(r, e); }
bool launch_plain_fixed_f32(const Request& r, hipError_t* e) { return launch_fixed<float>(r, e); }

}  // namespace sode
