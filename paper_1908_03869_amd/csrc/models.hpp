// models.hpp - drift and diffusion functors of the built-in SDE models.
//
// Each model supplies, for one orbit held in a per-lane array,
//   drift(n, t, p, y, f)     f_i(t, X, p) of Eq. (1) (the built-in models are
//                            autonomous and ignore t);
//   diffuse(n, t, p, y, xi)  overwrites xi with sum_j g_ij xi_j (diagonal
//                            noise: g_ij = 0 for i != j), without sqrt(dt);
//   noises(n)                m, the number of Wiener processes;
//   kStateNoise              whether g depends on the state; if it does,
//   dgdx(n, t, p, y, c)      c_i = g_ii dg_ii/dX_i, the coefficient of the
//                            Milstein correction (diagonal noise with g_ii a
//                            function of X_i alone).
// These are the two user functions of the paper's per-step integrator
// (Sec. 2.1.3, Step 4, Fig. 3), fixed at compile time instead of being
// assembled into a runtime-compiled source string.
#pragma once

#include "devmath.hpp"
#include "phase64.hpp"

namespace sode {

// sin of a phase difference: in binary64 the coupled kernels' sine
// (sin_phase64, accurate for |x| up to ~2^20; phases kept continuous, wrap 0,
// can drift far from [-pi, pi]) below 5e5, the library's beyond.
__device__ __forceinline__ float pair_sin(float x) { return dev_sin(x); }
__device__ __forceinline__ double pair_sin(double x) { return fabs(x) < 5e5 ? sin_phase64(x) : dev_sin(x); }

// Stochastic Kuramoto network, Eq. (5)/(6) of Sec. 2.2.1 with the
// parameter layout p = (K, omega_1..N, p_1..N) of that section's footnote:
// f_i = omega_i + (K/N) sum_j sin(theta_j - theta_i), g_ij = p_i delta_ij.
struct Kuramoto {
    static constexpr bool kStateNoise = false;
    static constexpr int kId = 0;
    __host__ __device__ static constexpr int noises(int n) { return n; }
    template <typename R>
    __device__ static void drift(int n, R, const R* __restrict__ p, const R* y, R* f)
    {
        const R scale = p[0] / (R)n;
        // Sizes compiled in (n a constant here): each unordered pair once,
        // sin(y_i - y_j) = -sin(y_j - y_i) exactly (the difference and both
        // sines are odd) and the j = i term is sin 0 = 0, with every sum
        // taking its terms in the order of j as below, so the results are
        // those of the loop over all pairs.  At a runtime n the arrays live
        // in scratch memory, where the second write per pair costs more than
        // the sine it saves: the loop over all pairs.
        if (__builtin_constant_p(n) && n <= 16) {
            for (int i = 0; i < n; ++i)
                f[i] = 0;
            for (int i = 0; i < n; ++i) {
                for (int j = i + 1; j < n; ++j) {
                    const R s = pair_sin(y[j] - y[i]);
                    f[i] += s;
                    f[j] -= s;
                }
                f[i] = f[i] * scale + p[1 + i];
            }
        } else {
            for (int i = 0; i < n; ++i) {
                const R yi = y[i];
                R coupling = 0;
                for (int j = 0; j < n; ++j)
                    coupling += pair_sin(y[j] - yi);
                f[i] = coupling * scale + p[1 + i];
            }
        }
    }
    template <typename R>
    __device__ static void diffuse(int n, R, const R* __restrict__ p, const R*, R* xi)
    {
        for (int i = 0; i < n; ++i)
            xi[i] = p[n + 1 + i] * xi[i];
    }
};

// The same Kuramoto drift through the angle-difference identity
//     sum_j sin(theta_j - theta_i) = cos(theta_i) S - sin(theta_i) C,
//     C = sum_j cos(theta_j),  S = sum_j sin(theta_j),
// which is exact in real arithmetic and costs O(N) instead of O(N^2)
// sines (the mean-field form of the coupling, Sec. 2.3.1).
struct KuramotoMeanField {
    static constexpr bool kStateNoise = false;
    static constexpr int kId = 0;
    __host__ __device__ static constexpr int noises(int n) { return n; }
    template <typename R>
    __device__ static void drift(int n, R, const R* __restrict__ p, const R* y, R* f)
    {
        R C = 0, S = 0;
        for (int j = 0; j < n; ++j) {
            C += dev_cos(y[j]);
            S += dev_sin(y[j]);
        }
        const R scale = p[0] / (R)n;
        for (int i = 0; i < n; ++i) {
            const R coupling = dev_cos(y[i]) * S - dev_sin(y[i]) * C;
            f[i] = coupling * scale + p[1 + i];
        }
    }
    template <typename R>
    __device__ static void diffuse(int n, R t, const R* __restrict__ p, const R* y, R* xi)
    {
        Kuramoto::diffuse(n, t, p, y, xi);
    }
};

// Ornstein-Uhlenbeck, dX_i = -a (X_i - mu) dt + s dW_i, p = (a, mu, s).
struct OrnsteinUhlenbeck {
    static constexpr bool kStateNoise = false;
    static constexpr int kId = 1;
    __host__ __device__ static constexpr int noises(int n) { return n; }
    template <typename R>
    __device__ static void drift(int n, R, const R* __restrict__ p, const R* y, R* f)
    {
        for (int i = 0; i < n; ++i)
            f[i] = -p[0] * (y[i] - p[1]);
    }
    template <typename R>
    __device__ static void diffuse(int n, R, const R* __restrict__ p, const R*, R* xi)
    {
        for (int i = 0; i < n; ++i)
            xi[i] = p[2] * xi[i];
    }
};

// Geometric Brownian motion, dX_i = mu X_i dt + s X_i dW_i, p = (mu, s).
struct GeometricBM {
    static constexpr bool kStateNoise = true;
    static constexpr int kId = 2;
    __host__ __device__ static constexpr int noises(int n) { return n; }
    template <typename R>
    __device__ static void drift(int n, R, const R* __restrict__ p, const R* y, R* f)
    {
        for (int i = 0; i < n; ++i)
            f[i] = p[0] * y[i];
    }
    template <typename R>
    __device__ static void diffuse(int n, R, const R* __restrict__ p, const R* y, R* xi)
    {
        for (int i = 0; i < n; ++i)
            xi[i] = p[1] * y[i] * xi[i];
    }
    template <typename R>
    __device__ static void dgdx(int n, R, const R* __restrict__ p, const R* y, R* c)
    {
        for (int i = 0; i < n; ++i)
            c[i] = (p[1] * y[i]) * p[1];
    }
};

// FitzHugh-Nagumo chain of N = n/2 units, state (v_1..v_N, w_1..w_N),
// p = (a, b, eps, D, sigma):
//   dv_i = [v_i - v_i^3/3 - w_i + D (v_{i-1} - 2 v_i + v_{i+1})] dt + sigma dW_i
//   dw_i = eps (v_i + a - b w_i) dt
// with no-flux ends (v_0 = v_1, v_{N+1} = v_N); noise on v only, m = N.
struct FhnChain {
    static constexpr bool kStateNoise = false;
    static constexpr int kId = 3;
    __host__ __device__ static constexpr int noises(int n) { return n / 2; }
    template <typename R>
    __device__ static void drift(int n, R, const R* __restrict__ p, const R* y, R* f)
    {
        const int N = n / 2;
        const R a = p[0], b = p[1], eps = p[2], D = p[3];
        for (int i = 0; i < N; ++i) {
            const R v = y[i];
            const R left = y[i > 0 ? i - 1 : 0];
            const R right = y[i < N - 1 ? i + 1 : N - 1];
            f[i] = v - v * v * v / (R)3 - y[N + i] + D * (left - (R)2 * v + right);
            f[N + i] = eps * (v + a - b * y[N + i]);
        }
    }
    template <typename R>
    __device__ static void diffuse(int n, R, const R* __restrict__ p, const R*, R* xi)
    {
        const int N = n / 2;
        for (int i = 0; i < N; ++i)
            xi[i] = p[4] * xi[i];
        for (int i = N; i < n; ++i)
            xi[i] = 0;
    }
};

// Dense random recurrent network, dX = (-X + W tanh X + b) dt + sigma dW,
// p = (W row-major n x n, b_1..n, sigma).
struct DenseRnn {
    static constexpr bool kStateNoise = false;
    static constexpr int kId = 4;
    __host__ __device__ static constexpr int noises(int n) { return n; }
    template <typename R>
    __device__ static void drift(int n, R, const R* __restrict__ p, const R* y, R* f)
    {
        const R* W = p;
        const R* bias = p + (size_t)n * n;
        for (int i = 0; i < n; ++i) {
            R acc = 0;
            for (int j = 0; j < n; ++j)
                acc += W[(size_t)i * n + j] * dev_tanh(y[j]);
            f[i] = -y[i] + acc + bias[i];
        }
    }
    template <typename R>
    __device__ static void diffuse(int n, R, const R* __restrict__ p, const R*, R* xi)
    {
        const R sigma = p[(size_t)n * n + n];
        for (int i = 0; i < n; ++i)
            xi[i] = sigma * xi[i];
    }
};

}  // namespace sode
