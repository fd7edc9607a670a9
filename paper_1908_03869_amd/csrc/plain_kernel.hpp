// plain_kernel.hpp - the one-orbit-per-lane stepper, shared by the built-in
// models (plain.hip) and by models given as source text, which are compiled
// at run time against this same header (rtc.cpp).
//
// This is the paper's own mapping (Sec. 2.1.3, Step 2, Fig. 1: one work-item
// integrates one orbit with private state arrays) written for gfx950.  All
// steps run inside one launch and every saved state goes straight to HBM
// (unlike the host loop of Sec. 2.1.4).
#pragma once

#include "devmath.hpp"
#include "kinds.hpp"
#include "noise.hpp"

namespace sode {

template <typename R>
struct PlainArgs {
    const R* __restrict__ X0;
    const R* __restrict__ p;
    R* __restrict__ out;
    const uint32_t* __restrict__ ids;
    const uint64_t* __restrict__ seeds;
    int n, m, d, p_per_orbit, observable;
    int wrap;  // Kuramoto phases: reduced to [-pi, pi] at the start and after every step
    int64_t orbits, stride, nsave;
    R t0, dt, sqdt;
    uint64_t seed, orbit_offset, step_offset;
    int* nonfinite;  // raised when a saved value is NaN or infinite (may be null)
};

template <typename R>
__device__ __forceinline__ R plain_order_parameter(int n, const R* y)
{
    R c = 0, s = 0;
    for (int j = 0; j < n; ++j) {
        c += dev_cos(y[j]);
        s += dev_sin(y[j]);
    }
    return dev_sqrt(c * c + s * s) / (R)n;
}

template <typename R>
__device__ __forceinline__ void plain_save(const PlainArgs<R>& a, int n, const R* y, R* dst)
{
    if (a.observable == kKuramotoR) {
        const R r = plain_order_parameter(n, y);
        note_nonfinite(a.nonfinite, r);
        dst[0] = r;
    } else {
        for (int i = 0; i < n; ++i) {
            note_nonfinite(a.nonfinite, y[i]);
            dst[i] = y[i];
        }
    }
}

template <typename R>
struct Eps;
template <>
struct Eps<double> {
    static constexpr double value = 0x1p-52;
};
template <>
struct Eps<float> {
    static constexpr float value = 0x1p-23f;
};

// Solve A x = b in place (A is n x n row-major with row pitch C; b becomes
// x) by Gaussian elimination with partial pivoting.
template <typename R, int C>
__device__ __forceinline__ void solve_dense(int n, R* A, R* b)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        R best = dev_fabs(A[col * C + col]);
        for (int r = col + 1; r < n; ++r) {
            const R v = dev_fabs(A[r * C + col]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        // Swap rows col and piv.  Written as a pass over the candidate rows
        // that selects values, with every load and store unconditional, so
        // that every index is known once the loops unroll and no address
        // depends on the pivot (a fixed n keeps A in registers); the rows
        // exchanged are the same.
        for (int r = col + 1; r < n; ++r) {
            const bool sw = r == piv;
            for (int c = 0; c < n; ++c) {
                const R top = A[col * C + c], row = A[r * C + c];
                A[col * C + c] = sw ? row : top;
                A[r * C + c] = sw ? top : row;
            }
            const R tb = b[col], rb = b[r];
            b[col] = sw ? rb : tb;
            b[r] = sw ? tb : rb;
        }
        for (int r = col + 1; r < n; ++r) {
            const R l = A[r * C + col] / A[col * C + col];
            for (int c = col; c < n; ++c)
                A[r * C + c] = A[r * C + c] - l * A[col * C + c];
            b[r] = b[r] - l * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        R acc = b[r];
        for (int c = r + 1; c < n; ++c)
            acc = acc - A[r * C + c] * b[c];
        b[r] = acc / A[r * C + r];
    }
}

// One step of a one-stage implicit Runge-Kutta method on the ODE limit
// g = 0 (the implicit solvers of Sec. 1.5; the implicit midpoint rule is the
// one the authors' earlier stiff-model work used, Sec. 3):
//     Y = X + dt f(t + c dt, X + c (Y - X)),
// c = 1 implicit Euler, c = 1/2 implicit midpoint.  Newton's method on
// G(Y) = Y - X - dt f(t + c dt, Z), Z = X + c (Y - X), from Y = X (the first
// iterate is the linearly implicit step); the Jacobian of f at Z by forward
// differences with step sqrt(eps) max(1, |Z_j|) (the step actually taken is
// re-read from the rounded Z_j + h); stop when the largest correction is at
// most 64 eps (1 + max |Y|).  After 50 iterations without convergence the
// state becomes NaN (every lane exits the loop).
template <class Model, typename R, int C>
__device__ __forceinline__ void implicit_step(int n, R t, R dt, R c, const R* __restrict__ p, R* X)
{
    const R eps = Eps<R>::value;
    const R sqeps = dev_sqrt(eps);
    R Y[C], Z[C], fz[C], fh[C], delta[C], A[C * C];
    for (int i = 0; i < n; ++i)
        Y[i] = X[i];
    const R ts = t + c * dt;
    bool converged = false;
    for (int it = 0; it < 50; ++it) {
        for (int i = 0; i < n; ++i)
            Z[i] = X[i] + c * (Y[i] - X[i]);
        Model::drift(n, ts, p, Z, fz);
        for (int j = 0; j < n; ++j) {
            const R zj = Z[j];
            R h = sqeps * (dev_fabs(zj) > (R)1 ? dev_fabs(zj) : (R)1);
            Z[j] = zj + h;
            h = Z[j] - zj;
            Model::drift(n, ts, p, Z, fh);
            Z[j] = zj;
            for (int i = 0; i < n; ++i)
                A[i * C + j] = (i == j ? (R)1 : (R)0) - c * dt * ((fh[i] - fz[i]) / h);
        }
        for (int i = 0; i < n; ++i)
            delta[i] = -(Y[i] - X[i] - dt * fz[i]);
        solve_dense<R, C>(n, A, delta);
        R dmax = 0, ymax = 0;
        for (int i = 0; i < n; ++i) {
            Y[i] = Y[i] + delta[i];
            dmax = dev_fabs(delta[i]) > dmax ? dev_fabs(delta[i]) : dmax;
            ymax = dev_fabs(Y[i]) > ymax ? dev_fabs(Y[i]) : ymax;
        }
        if (dmax <= (R)64 * eps * ((R)1 + ymax)) {
            converged = true;
            break;
        }
    }
    for (int i = 0; i < n; ++i)
        X[i] = converged ? Y[i] : __builtin_nan("");
}

// Body of the one-orbit-per-lane kernel (64-lane blocks).  NC > 0: the state
// dimension is the compile-time constant NC; NC == 0: the runtime a.n (up to
// kPlainMaxN, kImplicitMaxN for the implicit methods).  METH: Euler-Maruyama
// (Eq. 2); Milstein for diagonal state-dependent noise (the order-one method
// named as the next step in Sec. 1.5 and Sec. 4: the EM increment plus
// (1/2) g_ii dg_ii/dX_i ((dW_i)^2 - dt), dW_i = sqrt(dt) xi_i); the classical
// Runge-Kutta scheme on the drift alone (ODE limit); or an implicit step.
// t_k = t0 + k dt with k the step within this call.  MC: capacity of the
// noise array when a model has more Wiener processes than equations (0: the
// state capacity).
template <class Model, typename R, int NC, int METH, int MAXN, int MC = 0>
__device__ __forceinline__ void plain_body(const PlainArgs<R>& a)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= a.orbits)
        return;
    constexpr int CAP = NC > 0 ? NC : MAXN;
    constexpr int ICAP = NC > 0 ? NC : (MAXN < kImplicitMaxN ? MAXN : kImplicitMaxN);
    constexpr int XCAP = MC > CAP ? MC : CAP;
    const int n = NC > 0 ? NC : a.n;
    const int m = a.m;
    const int q = a.observable == kKuramotoR ? 1 : n;
    const R* __restrict__ p = a.p + (a.p_per_orbit ? o * (int64_t)a.d : 0);
    R* __restrict__ out = a.out + o * a.nsave * q;

    R y[CAP];
    for (int i = 0; i < n; ++i)
        y[i] = a.wrap ? dev_wrap_phase(a.X0[o * n + i]) : a.X0[o * n + i];
    plain_save(a, n, y, out);

    const Stream st = orbit_stream(o, a.seed, a.orbit_offset, a.ids, a.seeds);
    int64_t k = 0;
    for (int64_t s = 1; s < a.nsave; ++s) {
        for (int64_t kk = 0; kk < a.stride; ++kk, ++k) {
            const R t = a.t0 + (R)k * a.dt;
            if constexpr (METH == kEM) {
                // Euler-Maruyama, Eq. (2): X += f dt + (G xi) sqrt(dt).
                R f[CAP], xi[XCAP];
                Model::drift(n, t, p, y, f);
                normals<R>(st, (uint32_t)(a.step_offset + (uint64_t)k), m, xi);
                for (int j = m; j < n; ++j)
                    xi[j] = 0;
                Model::diffuse(n, t, p, y, xi);
                // The phase reduction (below for the other methods) in the
                // same pass: with a run-time n the state lives in scratch
                // memory, and a second pass over it costs a visible share
                // of a step.
                for (int i = 0; i < n; ++i) {
                    const R v = y[i] + f[i] * a.dt + xi[i] * a.sqdt;
                    y[i] = a.wrap ? dev_wrap_phase(v) : v;
                }
            } else if constexpr (METH == kMilstein) {
                R f[CAP], xi[XCAP], gxi[XCAP], c[CAP];
                Model::drift(n, t, p, y, f);
                Model::dgdx(n, t, p, y, c);
                normals<R>(st, (uint32_t)(a.step_offset + (uint64_t)k), m, xi);
                for (int j = m; j < n; ++j)
                    xi[j] = 0;
                for (int i = 0; i < (m > n ? m : n); ++i)
                    gxi[i] = xi[i];
                Model::diffuse(n, t, p, y, gxi);
                for (int i = 0; i < n; ++i) {
                    const R dW = a.sqdt * xi[i];
                    y[i] = y[i] + f[i] * a.dt + gxi[i] * a.sqdt;
                    y[i] = y[i] + (R)0.5 * c[i] * (dW * dW - a.dt);
                }
            } else if constexpr (METH == kRK4) {
                // Classical RK4 on dX = f dt.
                R kst[CAP], ksum[CAP], yt[CAP];
                const R h = a.dt, half = a.dt / (R)2;
                Model::drift(n, t, p, y, kst);
                for (int i = 0; i < n; ++i) {
                    ksum[i] = kst[i];
                    yt[i] = y[i] + half * kst[i];
                }
                Model::drift(n, t + half, p, yt, kst);
                for (int i = 0; i < n; ++i) {
                    ksum[i] += (R)2 * kst[i];
                    yt[i] = y[i] + half * kst[i];
                }
                Model::drift(n, t + half, p, yt, kst);
                for (int i = 0; i < n; ++i) {
                    ksum[i] += (R)2 * kst[i];
                    yt[i] = y[i] + h * kst[i];
                }
                Model::drift(n, t + h, p, yt, kst);
                for (int i = 0; i < n; ++i)
                    y[i] = y[i] + (h / (R)6) * (ksum[i] + kst[i]);
            } else {
                static_assert(METH == kImplicitEuler || METH == kImplicitMidpoint, "method");
                const R c = METH == kImplicitEuler ? (R)1 : (R)0.5;
                implicit_step<Model, R, ICAP>(n, t, a.dt, c, p, y);
            }
            if (METH != kEM && a.wrap) {  // the drift is 2 pi periodic in every phase
                for (int i = 0; i < n; ++i)
                    y[i] = dev_wrap_phase(y[i]);
            }
        }
        plain_save(a, n, y, out + s * q);
    }
}

}  // namespace sode
