// plain_implicit.hip - the implicit ODE steppers (implicit Euler, implicit
// midpoint) of the one-orbit-per-lane kernel for the built-in models, with
// the state dimension a runtime value up to kImplicitMaxN.  Kept apart from
// plain.hip because each lane's Newton matrix makes these instantiations
// large.
#include "launch.hpp"
#include "models.hpp"
#include "plain_kernel.hpp"

namespace sode {
namespace {

template <class Model, typename R, int METH>
__global__ __launch_bounds__(64) void plain_implicit_kernel(const PlainArgs<R> a)
{
    plain_body<Model, R, 0, METH, kImplicitMaxN>(a);
}

template <class Model, typename R>
hipError_t launch_model(const Request& r)
{
    const PlainArgs<R> a = plain_args<R>(r);
    const dim3 block(64);
    const dim3 grid((unsigned)((r.orbits + 63) / 64));
    if (r.method == kImplicitEuler)
        hipLaunchKernelGGL((plain_implicit_kernel<Model, R, kImplicitEuler>), grid, block, 0, r.stream, a);
    else
        hipLaunchKernelGGL((plain_implicit_kernel<Model, R, kImplicitMidpoint>), grid, block, 0, r.stream, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_implicit(const Request& r)
{
    if (r.n > kImplicitMaxN)
        return hipErrorInvalidValue;
    // Small systems: the fixed-size kernels (registers instead of private
    // memory, the same results bit for bit).
    hipError_t e = hipSuccess;
    const bool euler = r.method == kImplicitEuler;
    const bool fixed = sizeof(R) == 8 ? (euler ? launch_implicit_fixed_f64_euler(r, &e)
                                               : launch_implicit_fixed_f64_midpoint(r, &e))
                                      : (euler ? launch_implicit_fixed_f32_euler(r, &e)
                                               : launch_implicit_fixed_f32_midpoint(r, &e));
    if (fixed)
        return e;
    switch (r.model) {
    case kKuramoto:
        return r.drift == 1 ? launch_model<KuramotoMeanField, R>(r) : launch_model<Kuramoto, R>(r);
    case kOU: return launch_model<OrnsteinUhlenbeck, R>(r);
    case kGBM: return launch_model<GeometricBM, R>(r);
    case kFHN: return launch_model<FhnChain, R>(r);
    case kRNN: return launch_model<DenseRnn, R>(r);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_plain_implicit_f64(const Request& r) { return launch_implicit<double>(r); }
hipError_t launch_plain_implicit_f32(const Request& r) { return launch_implicit<float>(r); }

}  // namespace sode
