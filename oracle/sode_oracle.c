/*
 * sode_oracle.c - FP64 reference integrator for many independent orbits of an
 * Ito SDE system (Avramidis, Lalik & Akman, "SODECL", arXiv 1908.03869).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plainly written CPU definition
 * that the HIP library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it; the library never
 * does, and this file shares no code, header or constant table with the HIP
 * sources.
 *
 * Build flags: -O2 -ffp-contract=off, no fast-math, glibc libm.  Single
 * threaded.  Every sum runs in index order.  All arithmetic is IEEE binary64.
 *
 * Conventions fixed here where the paper is silent:
 *   - the uniform generator is Philox-4x32 with 10 rounds, the counter-based
 *     family the noise-generator section cites (Salmon et al. 2011);
 *   - counter = (global step k, orbit id, noise block b, tag 0),
 *     key = (seed mod 2^32, seed >> 32);
 *   - U1 = ((x0 >> 8) + 1) * 2^-24 in (0,1],  U2 = (x1 >> 8) * 2^-24 in [0,1);
 *   - words (x0,x1) give normals 4b and 4b+1 (cos first), (x2,x3) give 4b+2
 *     and 4b+3; normals with index >= m are dropped;
 *   - X^0 = X0 at t0 (0-based re-indexing of Eq. 2), t_k = t0 + k*dt;
 *   - out[o][s] = observable(X^{s*stride}) for s = 0..nsteps/stride, so the
 *     initial state is saved first.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { M_KURAMOTO = 0, M_OU = 1, M_GBM = 2, M_FHN = 3, M_RNN = 4 };
enum {
    METHOD_EM = 0,
    METHOD_RK4 = 1,
    METHOD_MILSTEIN = 2,
    METHOD_IMPLICIT_EULER = 3,
    METHOD_IMPLICIT_MIDPOINT = 4
};
enum { OBS_STATE = 0, OBS_KURAMOTO_R = 1 };

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), the counter-based
 * generator family behind the Random123 library that the noise-generator
 * section (Sec. 2.1.2) names.  One round: two 32x32->64 products of the
 * even counter words with the published multipliers, then a word shuffle
 * that XORs the high halves with the odd words and the key.  The key is
 * advanced by the published Weyl increments between rounds.               */
static const uint32_t PHILOX_MA = 0xD2511F53u; /* multiplies word 0 */
static const uint32_t PHILOX_MB = 0xCD9E8D57u; /* multiplies word 2 */
static const uint32_t WEYL_A = 0x9E3779B9u;    /* key word 0 increment */
static const uint32_t WEYL_B = 0xBB67AE85u;    /* key word 1 increment */

void oracle_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WEYL_A;
            k1 += WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHILOX_MA * (uint64_t)c[0];
        uint64_t prod_b = (uint64_t)PHILOX_MB * (uint64_t)c[2];
        uint32_t next[4];
        next[0] = (uint32_t)(prod_b >> 32) ^ c[1] ^ k0;
        next[1] = (uint32_t)prod_b;
        next[2] = (uint32_t)(prod_a >> 32) ^ c[3] ^ k1;
        next[3] = (uint32_t)prod_a;
        memcpy(c, next, sizeof c);
    }
    memcpy(out, c, sizeof c);
}

/* ------------------------------------------------------------------------ */
/* Box-Muller transform, Eq. (3) of Sec. 2.1.2: two uniforms give two
 * independent standard normals, the cosine branch first.  The uniforms are
 * 24-bit so that they are exact in binary32 as well as binary64; U1 excludes
 * zero so that the logarithm is finite.                                      */
void oracle_box_muller(uint32_t w0, uint32_t w1, double out[2])
{
    const double two_m24 = 1.0 / 16777216.0;
    double u1 = (double)((w0 >> 8) + 1u) * two_m24;
    double u2 = (double)(w1 >> 8) * two_m24;
    double radius = sqrt(-2.0 * log(u1));
    double angle = 2.0 * M_PI * u2;
    out[0] = radius * cos(angle);
    out[1] = radius * sin(angle);
}

/* The m standard normals N_j(0,1) that Eq. (2) consumes at global step k of
 * one orbit.  Eq. (3) is applied repeatedly when m > 2 (Sec. 2.1.2); each
 * Philox block supplies four words, hence two Box-Muller pairs.              */
void oracle_normals(uint64_t seed, uint32_t orbit_id, uint32_t step, int32_t m, double* xi)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int32_t nblocks = (m + 3) / 4;
    for (int32_t b = 0; b < nblocks; ++b) {
        uint32_t ctr[4] = {step, orbit_id, (uint32_t)b, 0u};
        uint32_t w[4];
        double pair[2];
        oracle_philox(ctr, key, w);
        for (int half = 0; half < 2; ++half) {
            oracle_box_muller(w[2 * half], w[2 * half + 1], pair);
            for (int q = 0; q < 2; ++q) {
                int32_t j = 4 * b + 2 * half + q;
                if (j < m)
                    xi[j] = pair[q];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Model dimensions (n equations, m noise terms, d parameters).               */
int oracle_model_dims_ok(int32_t model, int32_t n, int32_t m, int32_t d)
{
    if (n <= 0 || m <= 0 || d <= 0)
        return 0;
    switch (model) {
    case M_KURAMOTO: /* p = (K, omega_1..N, p_1..N), footnote of Sec. 2.2.1 */
        return m == n && d == 2 * n + 1;
    case M_OU: /* p = (a, mu, s) */
        return m == n && d == 3;
    case M_GBM: /* p = (mu, s) */
        return m == n && d == 2;
    case M_FHN: /* state (v_1..v_N, w_1..w_N), p = (a, b, eps, D, sigma) */
        return n % 2 == 0 && m == n / 2 && d == 5;
    case M_RNN: /* p = (W row-major N x N, b_1..N, sigma) */
        return m == n && (int64_t)d == (int64_t)n * n + n + 1;
    default:
        return 0;
    }
}

/* Drift f_i(t, X, p) of Eq. (1).
 *  Kuramoto: Eq. (5)/(6) with the parameter layout of the footnote of
 *    Sec. 2.2.1 and the loop of Fig. 5: the sum of sin(X_j - X_i) over every
 *    j (j = i included) in index order, scaled by K/N, plus omega_i.
 *  OU: -a (X_i - mu).   GBM: mu X_i.
 *  FHN chain: v' = v - v^3/3 - w + D (v_{i-1} - 2 v_i + v_{i+1}) with
 *    no-flux ends, w' = eps (v + a - b w).
 *  RNN: -X + W tanh(X) + b.                                                  */
void oracle_drift(int32_t model, int32_t n, int32_t m, int32_t d, double t,
                  const double* X, const double* p, double* f)
{
    (void)t;
    (void)m;
    (void)d;
    switch (model) {
    case M_KURAMOTO: {
        double K = p[0];
        for (int32_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int32_t j = 0; j < n; ++j)
                acc = acc + sin(X[j] - X[i]);
            acc = acc * (K / (double)n);
            f[i] = acc + p[1 + i];
        }
        break;
    }
    case M_OU:
        for (int32_t i = 0; i < n; ++i)
            f[i] = -p[0] * (X[i] - p[1]);
        break;
    case M_GBM:
        for (int32_t i = 0; i < n; ++i)
            f[i] = p[0] * X[i];
        break;
    case M_FHN: {
        int32_t N = n / 2;
        double a = p[0], b = p[1], eps = p[2], D = p[3];
        const double* v = X;
        const double* w = X + N;
        for (int32_t i = 0; i < N; ++i) {
            double left = v[i > 0 ? i - 1 : 0];
            double right = v[i < N - 1 ? i + 1 : N - 1];
            double lap = left - 2.0 * v[i] + right;
            f[i] = v[i] - v[i] * v[i] * v[i] / 3.0 - w[i] + D * lap;
            f[N + i] = eps * (v[i] + a - b * w[i]);
        }
        break;
    }
    case M_RNN: {
        const double* W = p;
        const double* bias = p + (size_t)n * n;
        double* th = (double*)malloc(sizeof(double) * (size_t)n);
        for (int32_t j = 0; j < n; ++j)
            th[j] = tanh(X[j]);
        for (int32_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int32_t j = 0; j < n; ++j)
                acc = acc + W[(size_t)i * n + j] * th[j];
            f[i] = -X[i] + acc + bias[i];
        }
        free(th);
        break;
    }
    default:
        break;
    }
}

/* Diffusion term sum_j g_ij(t, X, p) N_j of Eq. (1)/(2), without the
 * sqrt(dt) factor, which the stepper applies (Eq. 2).  All models here have
 * diagonal noise.  Kuramoto: g_ij = p_i delta_ij with p_i stored after the
 * frequencies (Fig. 5, sode_system_stoch).                                   */
void oracle_diffusion(int32_t model, int32_t n, int32_t m, int32_t d, double t,
                      const double* X, const double* p, const double* xi, double* gx)
{
    (void)t;
    switch (model) {
    case M_KURAMOTO:
        for (int32_t i = 0; i < n; ++i)
            gx[i] = p[d - m + i] * xi[i];
        break;
    case M_OU:
        for (int32_t i = 0; i < n; ++i)
            gx[i] = p[2] * xi[i];
        break;
    case M_GBM:
        for (int32_t i = 0; i < n; ++i)
            gx[i] = p[1] * X[i] * xi[i];
        break;
    case M_FHN: {
        int32_t N = n / 2;
        for (int32_t i = 0; i < N; ++i) {
            gx[i] = p[4] * xi[i];
            gx[N + i] = 0.0;
        }
        break;
    }
    case M_RNN:
        for (int32_t i = 0; i < n; ++i)
            gx[i] = p[d - 1] * xi[i];
        break;
    default:
        break;
    }
}

/* For the Milstein scheme: c_i = g_ii(X) * dg_ii/dX_i for each component.
 * Every model here has diagonal noise whose i-th coefficient depends on X_i
 * alone (or on nothing), the commutative case in which the order-one
 * scheme needs no iterated integrals beyond (dW_i)^2.  Only geometric
 * Brownian motion has a state-dependent coefficient, g_ii = s X_i.          */
void oracle_diffusion_dgdx(int32_t model, int32_t n, int32_t m, int32_t d, double t,
                           const double* X, const double* p, double* c)
{
    (void)m; (void)d; (void)t;
    for (int32_t i = 0; i < n; ++i)
        c[i] = model == M_GBM ? (p[1] * X[i]) * p[1] : 0.0;
}

/* Complex order parameter of Eq. (7), Sec. 2.3.1: r = |(1/N) sum_j e^{i theta_j}|. */
double oracle_order_parameter(int32_t n, const double* theta)
{
    double c = 0.0, s = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        c = c + cos(theta[j]);
        s = s + sin(theta[j]);
    }
    return sqrt(c * c + s * s) / (double)n;
}

static void save_observable(int32_t observable, int32_t n, const double* X, double* dst)
{
    if (observable == OBS_KURAMOTO_R)
        dst[0] = oracle_order_parameter(n, X);
    else
        for (int32_t i = 0; i < n; ++i)
            dst[i] = X[i];
}

/* ------------------------------------------------------------------------ */
/* A system as the integrator sees it: sizes and the three model functions
 * (drift f, diffusion G xi, and g_ii dg_ii/dX_i for Milstein).  Built-in
 * models go through the switch functions above; a runtime-defined model
 * supplies its own (oracle_integrate_custom).                               */
typedef void (*drift_cb)(double t, const double* X, const double* p, double* f);
typedef void (*diffusion_cb)(double t, const double* X, const double* p, const double* xi,
                             double* gx);

struct oracle_system {
    int32_t model; /* built-in model id, or -1 for callbacks */
    int32_t n, m, d;
    drift_cb drift;
    diffusion_cb diffusion;
};

static void sys_drift(const struct oracle_system* s, double t, const double* X, const double* p,
                      double* f)
{
    if (s->model >= 0)
        oracle_drift(s->model, s->n, s->m, s->d, t, X, p, f);
    else
        s->drift(t, X, p, f);
}

static void sys_diffusion(const struct oracle_system* s, double t, const double* X,
                          const double* p, const double* xi, double* gx)
{
    if (s->model >= 0)
        oracle_diffusion(s->model, s->n, s->m, s->d, t, X, p, xi, gx);
    else if (s->diffusion)
        s->diffusion(t, X, p, xi, gx);
    else
        for (int32_t i = 0; i < s->n; ++i)
            gx[i] = 0.0;
}

static void sys_dgdx(const struct oracle_system* s, double t, const double* X, const double* p,
                     double* c)
{
    if (s->model >= 0)
        oracle_diffusion_dgdx(s->model, s->n, s->m, s->d, t, X, p, c);
    else
        for (int32_t i = 0; i < s->n; ++i)
            c[i] = 0.0;
}

/* Solve A x = b in place (A n x n row-major, overwritten; b becomes x) by
 * Gaussian elimination with partial pivoting.                                */
static void solve_dense(int32_t n, double* A, double* b)
{
    for (int32_t col = 0; col < n; ++col) {
        int32_t piv = col;
        for (int32_t r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col]))
                piv = r;
        if (piv != col) {
            for (int32_t c = 0; c < n; ++c) {
                double tmp = A[col * n + c];
                A[col * n + c] = A[piv * n + c];
                A[piv * n + c] = tmp;
            }
            double tb = b[col];
            b[col] = b[piv];
            b[piv] = tb;
        }
        for (int32_t r = col + 1; r < n; ++r) {
            double l = A[r * n + col] / A[col * n + col];
            for (int32_t c = col; c < n; ++c)
                A[r * n + c] = A[r * n + c] - l * A[col * n + c];
            b[r] = b[r] - l * b[col];
        }
    }
    for (int32_t r = n - 1; r >= 0; --r) {
        double acc = b[r];
        for (int32_t c = r + 1; c < n; ++c)
            acc = acc - A[r * n + c] * b[c];
        b[r] = acc / A[r * n + r];
    }
}

/* One step of an implicit one-stage Runge-Kutta method for the ODE limit
 * g = 0 (the implicit solvers of Sec. 1.5; the implicit midpoint rule is the
 * one the authors' earlier stiff-model work used, Sec. 3):
 *     Y = X + dt f(t + c dt, X + c (Y - X)),
 * c = 1 for implicit Euler, c = 1/2 for the implicit midpoint rule.  Y is
 * found by Newton's method on G(Y) = Y - X - dt f(t + c dt, Z),
 * Z = X + c (Y - X), starting from Y = X (so the first iterate is the
 * linearly implicit step, the usual start for stiff systems); the Jacobian
 * of f at Z is formed by forward differences with step sqrt(eps) max(1,
 * |Z_j|), and each Newton system I - c dt J is solved by Gaussian
 * elimination with partial pivoting.  Iteration stops when the largest
 * correction is at most 64 eps (1 + max |Y|) (eps = 2^-52).  X is
 * overwritten with Y, or with NaN if 50 iterations did not converge.        */
static void implicit_step(const struct oracle_system* s, double t, double dt, double c,
                          const double* p, double* X, double* Y, double* Z, double* fz,
                          double* fh, double* A, double* delta)
{
    const int32_t n = s->n;
    const double eps = 0x1p-52;
    for (int32_t i = 0; i < n; ++i)
        Y[i] = X[i];
    const double ts = t + c * dt;
    int converged = 0;
    for (int32_t it = 0; it < 50; ++it) {
        for (int32_t i = 0; i < n; ++i)
            Z[i] = X[i] + c * (Y[i] - X[i]);
        sys_drift(s, ts, Z, p, fz);
        for (int32_t j = 0; j < n; ++j) {
            double zj = Z[j];
            double h = sqrt(eps) * (fabs(zj) > 1.0 ? fabs(zj) : 1.0);
            Z[j] = zj + h;
            h = Z[j] - zj;
            sys_drift(s, ts, Z, p, fh);
            Z[j] = zj;
            for (int32_t i = 0; i < n; ++i)
                A[i * n + j] = (i == j ? 1.0 : 0.0) - c * dt * ((fh[i] - fz[i]) / h);
        }
        for (int32_t i = 0; i < n; ++i)
            delta[i] = -(Y[i] - X[i] - dt * fz[i]);
        solve_dense(n, A, delta);
        double dmax = 0.0, ymax = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            Y[i] = Y[i] + delta[i];
            if (fabs(delta[i]) > dmax)
                dmax = fabs(delta[i]);
            if (fabs(Y[i]) > ymax)
                ymax = fabs(Y[i]);
        }
        if (dmax <= 64.0 * eps * (1.0 + ymax)) {
            converged = 1;
            break;
        }
    }
    for (int32_t i = 0; i < n; ++i)
        X[i] = converged ? Y[i] : NAN;
}

/* ------------------------------------------------------------------------ */
/* Integrate every orbit.  Per orbit, the Euler-Maruyama recursion of Eq. (2)
 * (Sec. 2.1.1; one call of the per-step integrator of Fig. 2 per step), or,
 * for method RK4, the classical four-stage Runge-Kutta scheme applied to the
 * ODE limit g = 0 (Sec. 1.1 last sentence; Sec. 1.5 lists Runge-Kutta among
 * the ODE methods), or, for method MILSTEIN, the strong order-one Milstein
 * scheme the paper names as its next stochastic method (Sec. 1.5, Sec. 4):
 * the Euler-Maruyama increment plus (1/2) g_ii dg_ii/dX_i ((dW_i)^2 - dt)
 * with dW_i = sqrt(dt) N_i, for diagonal noise (Kloeden & Platen, Numerical
 * Solution of SDEs, Sec. 10.3), or, for IMPLICIT_EULER / IMPLICIT_MIDPOINT,
 * implicit_step above on the ODE limit.  The state is observed every
 * `stride` steps, the host loop of Sec. 2.1.4 (Eq. 4) with s = stride.
 *
 *   X0  [orbits][n]    p  [orbits][d] (p_per_orbit = 1) or [d] (= 0)
 *   out [orbits][nsteps/stride + 1][q], q = n (state) or 1 (Kuramoto r)
 *   orbit id of orbit o = orbit_ids[o], else orbit_offset + o;
 *   seed of orbit o     = orbit_seeds[o], else seed.
 * Returns 0, or -1 for an argument error.                                    */
static int integrate_system(const struct oracle_system* sys, const double* X0, const double* p,
                            int32_t p_per_orbit, int64_t orbits, double t0, double dt,
                            int64_t nsteps, int64_t stride, uint64_t seed, uint64_t orbit_offset,
                            uint64_t step_offset, const uint32_t* orbit_ids,
                            const uint64_t* orbit_seeds, int32_t method, int32_t observable,
                            double* out)
{
    const int32_t n = sys->n, m = sys->m, d = sys->d;
    if (orbits < 0 || nsteps < 0 || stride < 1 || nsteps % stride != 0 || method < METHOD_EM ||
        method > METHOD_IMPLICIT_MIDPOINT)
        return -1;
    if (observable == OBS_KURAMOTO_R && sys->model != M_KURAMOTO)
        return -1;
    if (step_offset + (uint64_t)nsteps > 4294967296ull)
        return -1;
    int64_t nsave = nsteps / stride + 1;
    int32_t q = observable == OBS_KURAMOTO_R ? 1 : n;
    double* X = (double*)malloc(sizeof(double) * (size_t)n);
    double* f = (double*)malloc(sizeof(double) * (size_t)n);
    double* gx = (double*)malloc(sizeof(double) * (size_t)n);
    double* xi = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double* k1 = (double*)malloc(sizeof(double) * (size_t)n);
    double* k2 = (double*)malloc(sizeof(double) * (size_t)n);
    double* k3 = (double*)malloc(sizeof(double) * (size_t)n);
    double* k4 = (double*)malloc(sizeof(double) * (size_t)n);
    double* Y = (double*)malloc(sizeof(double) * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double* A = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    const double sqdt = sqrt(dt);

    for (int64_t o = 0; o < orbits; ++o) {
        uint32_t id = orbit_ids ? orbit_ids[o] : (uint32_t)(orbit_offset + (uint64_t)o);
        uint64_t sd = orbit_seeds ? orbit_seeds[o] : seed;
        const double* po = p + (p_per_orbit ? (size_t)o * (size_t)d : 0);
        double* out_o = out + (size_t)o * (size_t)nsave * (size_t)q;
        memcpy(X, X0 + (size_t)o * (size_t)n, sizeof(double) * (size_t)n);
        save_observable(observable, n, X, out_o);

        for (int64_t k = 0; k < nsteps; ++k) {
            double t = t0 + (double)k * dt;
            if (method == METHOD_EM || method == METHOD_MILSTEIN) {
                sys_drift(sys, t, X, po, f);
                oracle_normals(sd, id, (uint32_t)(step_offset + (uint64_t)k), m, xi);
                sys_diffusion(sys, t, X, po, xi, gx);
                if (method == METHOD_MILSTEIN)
                    sys_dgdx(sys, t, X, po, c);
                for (int32_t i = 0; i < n; ++i)
                    X[i] = X[i] + f[i] * dt + gx[i] * sqdt;
                if (method == METHOD_MILSTEIN) {
                    for (int32_t i = 0; i < n; ++i) {
                        double dW = i < m ? sqdt * xi[i] : 0.0;
                        X[i] = X[i] + 0.5 * c[i] * (dW * dW - dt);
                    }
                }
            } else if (method == METHOD_RK4) {
                sys_drift(sys, t, X, po, k1);
                for (int32_t i = 0; i < n; ++i)
                    Y[i] = X[i] + 0.5 * dt * k1[i];
                sys_drift(sys, t + 0.5 * dt, Y, po, k2);
                for (int32_t i = 0; i < n; ++i)
                    Y[i] = X[i] + 0.5 * dt * k2[i];
                sys_drift(sys, t + 0.5 * dt, Y, po, k3);
                for (int32_t i = 0; i < n; ++i)
                    Y[i] = X[i] + dt * k3[i];
                sys_drift(sys, t + dt, Y, po, k4);
                for (int32_t i = 0; i < n; ++i)
                    X[i] = X[i] + (dt / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
            } else {
                const double cc = method == METHOD_IMPLICIT_EULER ? 1.0 : 0.5;
                implicit_step(sys, t, dt, cc, po, X, Y, k1, k2, k3, A, k4);
            }
            if ((k + 1) % stride == 0)
                save_observable(observable, n, X, out_o + (size_t)((k + 1) / stride) * (size_t)q);
        }
    }
    free(X); free(f); free(gx); free(xi);
    free(k1); free(k2); free(k3); free(k4); free(Y); free(c); free(A);
    return 0;
}

int oracle_integrate(int32_t model, int32_t n, int32_t m, int32_t d,
                     const double* X0, const double* p, int32_t p_per_orbit,
                     int64_t orbits, double t0, double dt, int64_t nsteps, int64_t stride,
                     uint64_t seed, uint64_t orbit_offset, uint64_t step_offset,
                     const uint32_t* orbit_ids, const uint64_t* orbit_seeds,
                     int32_t method, int32_t observable, double* out)
{
    if (!oracle_model_dims_ok(model, n, m, d))
        return -1;
    struct oracle_system sys = {model, n, m, d, NULL, NULL};
    return integrate_system(&sys, X0, p, p_per_orbit, orbits, t0, dt, nsteps, stride, seed,
                            orbit_offset, step_offset, orbit_ids, orbit_seeds, method, observable,
                            out);
}

/* The same integrator for a model given as two C functions (the analogue of
 * the user-written system functions the paper compiles at run time,
 * Sec. 2.1.3 and Fig. 5): drift(t, X, p, f) and diffusion(t, X, p, xi, gx),
 * the latter returning sum_j g_ij xi_j without sqrt(dt).  Milstein treats
 * such a model as having state-independent noise.                            */
int oracle_integrate_custom(int32_t n, int32_t m, int32_t d, drift_cb drift,
                            diffusion_cb diffusion, const double* X0, const double* p,
                            int32_t p_per_orbit, int64_t orbits, double t0, double dt,
                            int64_t nsteps, int64_t stride, uint64_t seed, uint64_t orbit_offset,
                            uint64_t step_offset, const uint32_t* orbit_ids,
                            const uint64_t* orbit_seeds, int32_t method, double* out)
{
    if (n < 1 || m < 0 || d < 0 || !drift || (m > 0 && !diffusion))
        return -1;
    struct oracle_system sys = {-1, n, m, d, drift, diffusion};
    return integrate_system(&sys, X0, p, p_per_orbit, orbits, t0, dt, nsteps, stride, seed,
                            orbit_offset, step_offset, orbit_ids, orbit_seeds, method, OBS_STATE,
                            out);
}

/* ------------------------------------------------------------------------ */
/* Pathwise gradient of the time-averaged order parameter of Kuramoto orbits.
 *
 * Parameter fitting is the paper's motivating use (Sec. 1.2); the objective
 * here is R = (1/W) sum_{k=lo..hi} r(X^k), W = hi - lo + 1, the order
 * parameter of Eq. (7) averaged over a window of Euler-Maruyama iterates
 * (Eq. 6).  With the noise held fixed (the same Philox stream), X^N is a
 * deterministic function of p, and R's exact derivative is obtained by the
 * discrete adjoint of the map X^{k+1} = Phi_k(X^k, p):
 *     lambda^N = w_N grad r(X^N)
 *     for k = N-1 .. 0:
 *         g      += (d Phi_k / d p)^T lambda^{k+1}
 *         lambda^k = (d Phi_k / d X)^T lambda^{k+1} + w_k grad r(X^k)
 * with w_k = 1/W inside the window and 0 outside.  For the Kuramoto map
 *     d Phi_i/d X_j = delta_ij + dt K/N [cos(X_j - X_i) - delta_ij sum_l cos(X_l - X_i)]
 *     d Phi_i/d K   = dt/N sum_j sin(X_j - X_i)
 *     d Phi_i/d omega_i = dt,   d Phi_i/d p_i = sqrt(dt) N_i
 *     d r/d X_j = (S cos X_j - C sin X_j) / (N |Z|),  Z = C + iS = sum_j e^{i X_j}
 * (0 when |Z| < 1e-30).  Every product is formed from these pairwise
 * expressions; the full trajectory and its normals are stored.
 *
 *   R              [orbits]      objective of each orbit
 *   grad_per_orbit [orbits][d]   dL/dR_o * dR_o/dp (may be NULL)
 *   grad           [d]           sum over orbits in index order
 * Returns 0, or -1 for an argument error.                                    */
int oracle_kuramoto_adjoint(int32_t n, const double* X0, const double* p, int32_t p_per_orbit,
                            int64_t orbits, double t0, double dt, int64_t nsteps,
                            int64_t win_lo, int64_t win_hi, uint64_t seed,
                            uint64_t orbit_offset, uint64_t step_offset,
                            const double* dL_dR, double* R, double* grad_per_orbit, double* grad)
{
    const int32_t m = n, d = 2 * n + 1;
    if (n <= 0 || orbits < 0 || nsteps < 0 || win_lo < 0 || win_hi < win_lo || win_hi > nsteps)
        return -1;
    (void)t0;
    const double W = (double)(win_hi - win_lo + 1);
    const double sqdt = sqrt(dt);
    double* traj = (double*)malloc(sizeof(double) * (size_t)(nsteps + 1) * (size_t)n);
    double* noise = (double*)malloc(sizeof(double) * (size_t)(nsteps > 0 ? nsteps : 1) * (size_t)m);
    double* f = (double*)malloc(sizeof(double) * (size_t)n);
    double* gx = (double*)malloc(sizeof(double) * (size_t)n);
    double* lam = (double*)malloc(sizeof(double) * (size_t)n);
    double* mu = (double*)malloc(sizeof(double) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)d);
    for (int32_t q = 0; q < d; ++q)
        grad[q] = 0.0;

    for (int64_t o = 0; o < orbits; ++o) {
        const double* po = p + (p_per_orbit ? (size_t)o * (size_t)d : 0);
        const double K = po[0];
        const uint32_t id = (uint32_t)(orbit_offset + (uint64_t)o);
        /* forward pass, storing every state and every normal */
        memcpy(traj, X0 + (size_t)o * (size_t)n, sizeof(double) * (size_t)n);
        for (int64_t k = 0; k < nsteps; ++k) {
            const double* X = traj + (size_t)k * (size_t)n;
            double* Xn = traj + (size_t)(k + 1) * (size_t)n;
            double* xi = noise + (size_t)k * (size_t)m;
            oracle_drift(M_KURAMOTO, n, m, d, t0 + (double)k * dt, X, po, f);
            oracle_normals(seed, id, (uint32_t)(step_offset + (uint64_t)k), m, xi);
            oracle_diffusion(M_KURAMOTO, n, m, d, t0 + (double)k * dt, X, po, xi, gx);
            for (int32_t i = 0; i < n; ++i)
                Xn[i] = X[i] + f[i] * dt + gx[i] * sqdt;
        }
        double Ro = 0.0;
        for (int64_t k = win_lo; k <= win_hi; ++k)
            Ro = Ro + oracle_order_parameter(n, traj + (size_t)k * (size_t)n);
        Ro = Ro / W;
        R[o] = Ro;

        /* reverse pass */
        for (int32_t q = 0; q < d; ++q)
            g[q] = 0.0;
        for (int32_t i = 0; i < n; ++i)
            lam[i] = 0.0;
        for (int64_t k = nsteps; k >= 0; --k) {
            const double* X = traj + (size_t)k * (size_t)n;
            if (k < nsteps) {
                const double* xi = noise + (size_t)k * (size_t)m;
                /* parameter sensitivities of Phi_k against lambda^{k+1} */
                for (int32_t i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int32_t j = 0; j < n; ++j)
                        s = s + sin(X[j] - X[i]);
                    g[0] = g[0] + lam[i] * (dt / (double)n) * s;
                    g[1 + i] = g[1 + i] + lam[i] * dt;
                    g[1 + n + i] = g[1 + n + i] + lam[i] * sqdt * xi[i];
                }
                /* lambda^k = (d Phi_k / d X)^T lambda^{k+1} */
                for (int32_t j = 0; j < n; ++j) {
                    double a = 0.0, b = 0.0;
                    for (int32_t i = 0; i < n; ++i) {
                        a = a + lam[i] * cos(X[j] - X[i]);
                        b = b + cos(X[i] - X[j]);
                    }
                    mu[j] = lam[j] + dt * (K / (double)n) * (a - lam[j] * b);
                }
                memcpy(lam, mu, sizeof(double) * (size_t)n);
            }
            if (k >= win_lo && k <= win_hi) {
                double c = 0.0, s = 0.0;
                for (int32_t j = 0; j < n; ++j) {
                    c = c + cos(X[j]);
                    s = s + sin(X[j]);
                }
                const double z = sqrt(c * c + s * s);
                if (z >= 1e-30)
                    for (int32_t j = 0; j < n; ++j)
                        lam[j] = lam[j] + (s * cos(X[j]) - c * sin(X[j])) / ((double)n * z) / W;
            }
        }
        const double wgt = dL_dR ? dL_dR[o] : 1.0;
        for (int32_t q = 0; q < d; ++q) {
            if (grad_per_orbit)
                grad_per_orbit[(size_t)o * (size_t)d + q] = wgt * g[q];
            grad[q] = grad[q] + wgt * g[q];
        }
    }
    free(traj); free(noise); free(f); free(gx); free(lam); free(mu); free(g);
    return 0;
}
