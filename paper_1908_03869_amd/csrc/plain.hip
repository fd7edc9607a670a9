// plain.hip - one orbit per lane, any built-in model, binary64 or binary32.
//
// This is the paper's own mapping (Sec. 2.1.3, Step 2, Fig. 1: one OpenCL
// work-item integrates one orbit with private state arrays) written directly
// for gfx950.  It serves three purposes: the FP64 path of small systems, the
// generic path for every model and size the specialised kernels do not
// cover, and the plain per-orbit FP64 baseline that the specialised kernels
// are measured against.  Unlike the paper's host loop (Sec. 2.1.4), all
// steps run inside one launch and every saved state goes straight to HBM.
#include "launch.hpp"
#include "models.hpp"
#include "noise.hpp"

namespace sode {
namespace {

template <typename R>
struct PlainArgs {
    const R* __restrict__ X0;
    const R* __restrict__ p;
    R* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int n, m, d, p_per_orbit, observable;
    int64_t orbits, stride, nsave;
    R t0, dt, sqdt;
    uint64_t seed, orbit_offset, step_offset;
};

template <typename R>
__device__ __forceinline__ R order_parameter(int n, const R* y)
{
    R c = 0, s = 0;
    for (int j = 0; j < n; ++j) {
        c += dev_cos(y[j]);
        s += dev_sin(y[j]);
    }
    return dev_sqrt(c * c + s * s) / (R)n;
}

template <typename R>
__device__ __forceinline__ void save(const PlainArgs<R>& a, int n, const R* y, R* dst)
{
    if (a.observable == kKuramotoR) {
        dst[0] = order_parameter(n, y);
    } else {
        for (int i = 0; i < n; ++i)
            dst[i] = y[i];
    }
}

// NC > 0: the state dimension is the compile-time constant NC; NC == 0: the
// runtime a.n (<= kPlainMaxN).  METH: Euler-Maruyama (Eq. 2), the Milstein
// scheme for diagonal state-dependent noise (the order-one method named as
// the next step in Sec. 1.5 and Sec. 4: the EM increment plus
// (1/2) g_ii dg_ii/dX_i ((dW_i)^2 - dt), dW_i = sqrt(dt) xi_i), or the
// classical Runge-Kutta scheme on the drift alone (ODE limit).
template <class Model, typename R, int NC, int METH>
__global__ __launch_bounds__(64) void plain_kernel(const PlainArgs<R> a)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= a.orbits)
        return;
    constexpr int CAP = NC > 0 ? NC : kPlainMaxN;
    const int n = NC > 0 ? NC : a.n;
    const int m = NC > 0 ? Model::noises(NC) : a.m;
    const int q = a.observable == kKuramotoR ? 1 : n;
    const R* __restrict__ p = a.p + (a.p_per_orbit ? o * (int64_t)a.d : 0);
    R* __restrict__ out = a.out + o * a.nsave * q;

    R y[CAP];
    for (int i = 0; i < n; ++i)
        y[i] = a.X0[o * n + i];
    save(a, n, y, out);

    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);
    int64_t k = 0;
    for (int64_t s = 1; s < a.nsave; ++s) {
        for (int64_t kk = 0; kk < a.stride; ++kk, ++k) {
            if constexpr (METH == kEM) {
                // Euler-Maruyama, Eq. (2): X += f dt + (G xi) sqrt(dt).
                R f[CAP], xi[CAP];
                Model::drift(n, p, y, f);
                normals<R>(st, (uint32_t)(a.step_offset + (uint64_t)k), m, xi);
                for (int j = m; j < n; ++j)
                    xi[j] = 0;
                Model::diffuse(n, p, y, xi);
                for (int i = 0; i < n; ++i)
                    y[i] = y[i] + f[i] * a.dt + xi[i] * a.sqdt;
            } else if constexpr (METH == kMilstein) {
                R f[CAP], xi[CAP], gxi[CAP], c[CAP];
                Model::drift(n, p, y, f);
                Model::dgdx(n, p, y, c);
                normals<R>(st, (uint32_t)(a.step_offset + (uint64_t)k), m, xi);
                for (int j = m; j < n; ++j)
                    xi[j] = 0;
                for (int i = 0; i < n; ++i)
                    gxi[i] = xi[i];
                Model::diffuse(n, p, y, gxi);
                for (int i = 0; i < n; ++i) {
                    const R dW = a.sqdt * xi[i];
                    y[i] = y[i] + f[i] * a.dt + gxi[i] * a.sqdt;
                    y[i] = y[i] + (R)0.5 * c[i] * (dW * dW - a.dt);
                }
            } else {
                // Classical RK4 on dX = f dt.
                R kst[CAP], ksum[CAP], yt[CAP];
                const R h = a.dt, half = a.dt / (R)2;
                Model::drift(n, p, y, kst);
                for (int i = 0; i < n; ++i) {
                    ksum[i] = kst[i];
                    yt[i] = y[i] + half * kst[i];
                }
                Model::drift(n, p, yt, kst);
                for (int i = 0; i < n; ++i) {
                    ksum[i] += (R)2 * kst[i];
                    yt[i] = y[i] + half * kst[i];
                }
                Model::drift(n, p, yt, kst);
                for (int i = 0; i < n; ++i) {
                    ksum[i] += (R)2 * kst[i];
                    yt[i] = y[i] + h * kst[i];
                }
                Model::drift(n, p, yt, kst);
                for (int i = 0; i < n; ++i)
                    y[i] = y[i] + (h / (R)6) * (ksum[i] + kst[i]);
            }
        }
        save(a, n, y, out + s * q);
    }
}

template <class Model, typename R, int NC>
hipError_t launch_one(const Request& r)
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
    a.orbits = r.orbits;
    a.stride = r.stride;
    a.nsave = r.nsave;
    a.t0 = (R)r.t0;
    a.dt = (R)r.dt;
    a.sqdt = (R)sqrt(r.dt);
    a.seed = r.seed;
    a.orbit_offset = r.orbit_offset;
    a.step_offset = r.step_offset;
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

template <typename R>
hipError_t launch_plain(const Request& r)
{
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
        return launch_one<OrnsteinUhlenbeck, R, 0>(r);
    case kGBM:
        if (r.n == 1)
            return launch_one<GeometricBM, R, 1>(r);
        return launch_one<GeometricBM, R, 0>(r);
    case kFHN:
        return launch_one<FhnChain, R, 0>(r);
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
