// plain.hip - one orbit per lane, any built-in model, binary64 or binary32.
//
// The stepper itself is in plain_kernel.hpp.  This kernel serves three
// purposes: the FP64 path of small systems, the generic path for every
// model, size and method the specialised kernels do not cover, and the plain
// per-orbit FP64 baseline that the specialised kernels are measured against.
#include "launch.hpp"
#include "models.hpp"
#include "plain_kernel.hpp"

namespace sode {
namespace {

template <class Model, typename R, int NC, int METH>
__global__ __launch_bounds__(64) void plain_kernel(const PlainArgs<R> a)
{
    plain_body<Model, R, NC, METH, kPlainMaxN>(a);
}

}  // namespace

template <typename R>
PlainArgs<R> plain_args(const Request& r)
{
    PlainArgs<R> a;
    a.X0 = static_cast<const R*>(r.X0);
    a.p = static_cast<const R*>(r.p);
    a.out = static_cast<R*>(r.out);
    a.ids = r.orbit_ids;
    a.seeds = r.orbit_seeds;
    a.n = r.n;
    a.m = r.m;
    a.d = r.d;
    a.p_per_orbit = r.p_per_orbit;
    a.observable = r.observable;
    a.wrap = r.model == kKuramoto && r.wrap ? 1 : 0;
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.t0 = (R)r.t0;
    a.dt = (R)r.dt;
    a.sqdt = (R)sqrt(r.dt);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
    a.nonfinite = r.nonfinite;
    return a;
}
template PlainArgs<double> plain_args<double>(const Request&);
template PlainArgs<float> plain_args<float>(const Request&);

namespace {

template <class Model, typename R, int NC>
hipError_t launch_one(const Request& r)
{
    const PlainArgs<R> a = plain_args<R>(r);
    const dim3 block(64);
    const dim3 grid((unsigned)((r.orbits + 63) / 64));
    if (r.method == kRK4)
        hipLaunchKernelGGL((plain_kernel<Model, R, NC, kRK4>), grid, block, 0, r.stream, a);
    else if (r.method == kMilstein && Model::kStateNoise)
        hipLaunchKernelGGL((plain_kernel<Model, R, NC, (Model::kStateNoise ? kMilstein : kEM)>),
                           grid, block, 0, r.stream, a);
    else  // EM; and Milstein with state-independent noise, where the correction is zero
        hipLaunchKernelGGL((plain_kernel<Model, R, NC, kEM>), grid, block, 0, r.stream, a);
    return hipGetLastError();
}

// The fixed-size kernel of plain_fixed.hip where there is one for r.n, else
// the runtime-n kernel.
template <class Model, typename R>
hipError_t launch_fixed_or(const Request& r)
{
    hipError_t e = hipSuccess;
    if (sizeof(R) == 8 ? launch_plain_fixed_f64(r, &e) : launch_plain_fixed_f32(r, &e))
        return e;
    return launch_one<Model, R, 0>(r);
}

template <typename R>
hipError_t launch_plain(const Request& r)
{
    if (r.method == kImplicitEuler || r.method == kImplicitMidpoint)
        return sizeof(R) == 8 ? launch_plain_implicit_f64(r) : launch_plain_implicit_f32(r);
    switch (r.model) {
    case kKuramoto:
        if (r.drift == 1) {
            switch (r.n) {
            case 4: return launch_one<KuramotoMeanField, R, 4>(r);
            case 5: return launch_one<KuramotoMeanField, R, 5>(r);
            case 10: return launch_one<KuramotoMeanField, R, 10>(r);
            case 15: return launch_one<KuramotoMeanField, R, 15>(r);
            default: return launch_one<KuramotoMeanField, R, 0>(r);
            }
        }
        switch (r.n) {
        case 4: return launch_one<Kuramoto, R, 4>(r);
        case 5: return launch_one<Kuramoto, R, 5>(r);
        case 10: return launch_one<Kuramoto, R, 10>(r);
        case 15: return launch_one<Kuramoto, R, 15>(r);
        default: return launch_one<Kuramoto, R, 0>(r);
        }
    case kOU:
        if (r.n == 1)
            return launch_one<OrnsteinUhlenbeck, R, 1>(r);
        return launch_fixed_or<OrnsteinUhlenbeck, R>(r);
    case kGBM:
        if (r.n == 1)
            return launch_one<GeometricBM, R, 1>(r);
        return launch_fixed_or<GeometricBM, R>(r);
    case kFHN:
        return launch_fixed_or<FhnChain, R>(r);
    case kRNN:
        return launch_one<DenseRnn, R, 0>(r);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_plain_f64(const Request& r) { return launch_plain<double>(r); }
hipError_t launch_plain_f32(const Request& r) { return launch_plain<float>(r); }

}  // namespace sode
