// implicit_fixed.hpp - the implicit Euler / implicit midpoint steppers of
// the one-orbit-per-lane kernel with the state dimension as a compile-time
// constant, for the small systems these methods are mostly used on (n = 1,
// 2, 3, 4, 6, 8).  With n known, every loop of the Newton iteration, the
// finite-difference Jacobian and the dense elimination unrolls and the
// per-lane vectors and matrix live in registers instead of private memory
// (the runtime-n kernel of plain_implicit.hip).  The arithmetic, and so the
// result, is the same bit for bit.  Each translation unit that includes this
// header instantiates one precision and one method.
#pragma once

#include "launch.hpp"
#include "models.hpp"
#include "plain_kernel.hpp"

namespace sode {

template <class Model, typename R, int NC, int METH>
__global__ __launch_bounds__(64) void plain_implicit_fixed_kernel(const PlainArgs<R> a)
{
    plain_body<Model, R, NC, METH, NC>(a);
}

template <class Model, typename R, int NC, int METH>
hipError_t launch_implicit_fixed_n(const Request& r)
{
    const PlainArgs<R> a = plain_args<R>(r);
    const dim3 grid((unsigned)((r.orbits + 63) / 64));
    hipLaunchKernelGGL((plain_implicit_fixed_kernel<Model, R, NC, METH>), grid, dim3(64), 0, r.stream, a);
    return hipGetLastError();
}

template <class Model, typename R, int METH>
bool launch_implicit_fixed_model(const Request& r, hipError_t* e)
{
    switch (r.n) {
    case 1: *e = launch_implicit_fixed_n<Model, R, 1, METH>(r); return true;
    case 2: *e = launch_implicit_fixed_n<Model, R, 2, METH>(r); return true;
    case 3: *e = launch_implicit_fixed_n<Model, R, 3, METH>(r); return true;
    case 4: *e = launch_implicit_fixed_n<Model, R, 4, METH>(r); return true;
    case 6: *e = launch_implicit_fixed_n<Model, R, 6, METH>(r); return true;
    case 8: *e = launch_implicit_fixed_n<Model, R, 8, METH>(r); return true;
    default: return false;
    }
}

// True if a fixed-size kernel took the request (its launch status in *e);
// false for sizes without one.
template <typename R, int METH>
bool launch_implicit_fixed(const Request& r, hipError_t* e)
{
    switch (r.model) {
    case kKuramoto:
        return r.drift == 1 ? launch_implicit_fixed_model<KuramotoMeanField, R, METH>(r, e)
                            : launch_implicit_fixed_model<Kuramoto, R, METH>(r, e);
    case kOU: return launch_implicit_fixed_model<OrnsteinUhlenbeck, R, METH>(r, e);
    case kGBM: return launch_implicit_fixed_model<GeometricBM, R, METH>(r, e);
    case kFHN:
        if (r.n % 2 != 0)
            return false;
        return launch_implicit_fixed_model<FhnChain, R, METH>(r, e);
    case kRNN: return launch_implicit_fixed_model<DenseRnn, R, METH>(r, e);
    default: return false;
    }
}

}  // namespace sode
