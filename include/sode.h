/*
 * sode.h - C ABI of libsode, an MI355X (gfx950) library that integrates many
 * independent orbits of an Ito SDE system at once (the problem of
 * Avramidis, Lalik & Akman, "SODECL", arXiv 1908.03869).
 *
 * The system is Eq. (1) of Sec. 1.1:
 *     dX_i = f_i(t, X, p) dt + sum_j g_ij(t, X, p) dW_j,   i = 1..n, j = 1..m,
 * with d parameters p.  Each orbit is one (X0, p, noise stream) triple; the
 * paper's Python interface (Table 2, Fig. 4) takes the same quantities:
 * initial states, parameter sets, solver, orbit count, n / d / m, dt, time
 * span and the number of steps between saved states.
 *
 * Conventions shared by every entry point:
 *   - Pointers to arrays are DEVICE pointers (HIP global memory), caller
 *     owned, contiguous and row-major.  The library never frees them.
 *   - Floating-point arrays (X0, p, out) have the handle's precision:
 *     float for precision 32, double for precision 64.
 *   - Launches are asynchronous on the HIP stream passed as `stream`
 *     (a hipStream_t; NULL = the default stream).  Argument errors are
 *     reported synchronously, before any HIP call is made; errors raised by
 *     the device surface at sode_sync() or at the next call on the handle.
 *   - A handle is not thread-safe; calls on one handle must be serialised.
 *   - Every function returns SODE_OK (0) or a negative sode_status.
 */
#ifndef SODE_H
#define SODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sode_ctx* sode_t; /* opaque, owned by the library */

/*
 * One instance of a ragged batch (sode_integrate_ragged): its own size,
 * length, save stride, noise stream and places in packed arrays.  64 bytes.
 */
typedef struct sode_instance {
    int32_t n;           /* state dimension of this instance (FHN: 2 x units) */
    int32_t reserved0;   /* must be 0 */
    int64_t nsteps;      /* >= 0, a multiple of stride, < 2^32 */
    int64_t stride;      /* >= 1: out holds X^0, X^stride, ..., X^nsteps */
    int64_t x0_offset;   /* element offset of X0_i [n] in the packed X0 */
    int64_t p_offset;    /* element offset of p_i [d] in the packed p */
    int64_t out_offset;  /* element offset of out_i [nsteps/stride + 1][n] in out */
    uint64_t seed;       /* Philox key of the instance */
    uint32_t orbit_id;   /* Philox counter word 1 of the instance */
    uint32_t reserved1;  /* must be 0 */
} sode_instance_t;

enum sode_status {
    SODE_OK = 0,
    SODE_EINVAL = -1,       /* invalid argument (shape, pointer, option)        */
    SODE_ENOMEM = -2,       /* allocation of library-owned memory failed        */
    SODE_EDEVICE = -3,      /* a HIP call or a kernel launch failed             */
    SODE_EUNSUPPORTED = -4, /* valid request that this build does not implement */
    SODE_ENONFINITE = -5,   /* a saved state was NaN or infinite                */
    SODE_EBUILD = -6,       /* run-time compilation of a model source failed    */
    SODE_ETOOBIG = -7       /* request exceeds a fixed, library-owned capacity   */
};

/*
 * sode_create - make a handle for one SDE model.
 *
 * model  "kuramoto": stochastic Kuramoto network, Eq. (5)/(6) of Sec. 2.2.1
 *                    (f_i = omega_i + K/N sum_j sin(theta_j - theta_i),
 *                    g_ij = p_i delta_ij); n = m = N, d = 2N+1,
 *                    p = (K, omega_1..N, p_1..N) (footnote of Sec. 2.2.1).
 *        "ou":       Ornstein-Uhlenbeck, dX_i = -a (X_i - mu) dt + s dW_i;
 *                    m = n, d = 3, p = (a, mu, s).
 *        "gbm":      geometric Brownian motion, dX_i = mu X_i dt + s X_i dW_i;
 *                    m = n, d = 2, p = (mu, s).
 *        "fhn":      FitzHugh-Nagumo chain of N = n/2 units, state
 *                    (v_1..v_N, w_1..w_N), dv_i = [v_i - v_i^3/3 - w_i +
 *                    D (v_{i-1} - 2 v_i + v_{i+1})] dt + sigma dW_i,
 *                    dw_i = eps (v_i + a - b w_i) dt, no-flux ends;
 *                    m = N, d = 5, p = (a, b, eps, D, sigma).
 *        "rnn":      dense random network, dX = (-X + W tanh X + b) dt +
 *                    sigma dW; m = n, d = n^2 + n + 1, p = (W row-major, b, sigma).
 * n, m, d must match the model, else SODE_EINVAL.  On success *out receives
 * a new handle with default options (precision 32, method EM, observable
 * "state", kernel auto, per-orbit parameters).  No HIP call is made.
 */
int sode_create(const char* model, int32_t n, int32_t m, int32_t d, sode_t* out);

/*
 * sode_create_custom - make a handle for a model given as source text: the
 * bodies of its two system functions, as the paper's users write the drift
 * and stochastic functions of their system (Sec. 2.1.3, Fig. 5) and the
 * framework compiles them at run time.
 *
 *   drift_body      C/C++ statements that set f[0..n) from
 *                       real t, const real* y, const real* p
 *                   (real is float or double after the handle's precision);
 *                   the device math functions (sin, cos, exp, tanh, sqrt,
 *                   pow, fabs, ...) are available.
 *   diffusion_body  statements that set gx[0..n) = sum_j g_ij(t, y, p) xi[j]
 *                   from t, y, p and const real* xi (m normals), without
 *                   sqrt(dt), which the stepper applies (Eq. 2).  May be
 *                   NULL when m = 0 (an ODE).
 *   n, m, d         1 <= n <= 128 equations, 0 <= m <= 128 Wiener
 *                   processes, d >= 0 parameters per orbit (p must still
 *                   be a valid pointer when d = 0).
 * The texts are copied; nothing is compiled here (no HIP call is made).  The
 * handle takes every option of sode_create's handles except observable r;
 * it runs on the one-orbit-per-lane stepper with methods 0 (EM), 1 (RK4),
 * 3 and 4 (implicit, n <= 16); method 2 gives SODE_EUNSUPPORTED (the
 * diffusion's state derivative is not known).  Noise addressing, saves,
 * sode_integrate_ex offsets and ids are those of the built-in models.
 * Compilation (hipRTC, gfx950) happens in sode_build or on the first
 * integrate call of each precision, and is cached per process by source.
 * Returns SODE_EINVAL for a NULL drift body, a NULL diffusion body with
 * m > 0 or sizes out of range.
 */
int sode_create_custom(const char* drift_body, const char* diffusion_body, int32_t n, int32_t m,
                       int32_t d, sode_t* out);

/*
 * sode_build - compile a source-text handle for its current precision now
 * (host work only: no GPU is needed).  SODE_OK, or SODE_EBUILD with the
 * compiler's messages in sode_build_log (line numbers refer to the drift or
 * diffusion body).  A handle of a built-in model returns SODE_OK.
 *
 * sode_build_log - copy the last compilation log into buf (at most len - 1
 * bytes and a terminating NUL; buf may be NULL); *needed (if not NULL)
 * receives the full length + 1.
 */
int sode_build(sode_t h);
int sode_build_log(sode_t h, char* buf, size_t len, size_t* needed);

/*
 * sode_set_option / sode_get_option - integer options of a handle.
 *
 *   "precision"    32 | 64   arithmetic type of the state and of X0/p/out.
 *   "method"       0 = Euler-Maruyama, Eq. (2) of Sec. 2.1.1 (default);
 *                  1 = classical RK4 on the ODE limit g = 0 (Sec. 1.1; the
 *                      Runge-Kutta ODE solver of Sec. 1.5): the diffusion is
 *                      ignored and no noise is drawn.  Every built-in model
 *                      has a diffusion, as has a source-text model with
 *                      m > 0: for those, integrate returns
 *                      SODE_EUNSUPPORTED unless "ode_limit" is 1;
 *                  2 = Milstein, the strong order-one scheme named as the
 *                      next stochastic method (Sec. 1.5, Sec. 4), for
 *                      diagonal noise: the EM increment plus
 *                      (1/2) g_ii dg_ii/dX_i ((dW_i)^2 - dt).  Plain kernel
 *                      only; for models whose diffusion does not depend on
 *                      the state (all but "gbm") it equals EM exactly;
 *                  3 = implicit Euler, 4 = implicit midpoint rule, on the
 *                      ODE limit g = 0 (the implicit solvers of Sec. 1.5):
 *                      Y = X + dt f(t + c dt, X + c (Y - X)), c = 1 or 1/2,
 *                      solved per step by Newton's method from Y = X with
 *                      a forward-difference Jacobian, stopping at a largest
 *                      correction of 64 eps (1 + max|Y|); a step that has
 *                      not converged after 50 iterations sets the state to
 *                      NaN.  Plain kernel only, n <= 16 (each lane holds an
 *                      n x n matrix); "ode_limit" as for RK4.
 *   "ode_limit"    0 (default) = RK4 and the implicit methods are refused
 *                  (SODE_EUNSUPPORTED) on a model with a diffusion;
 *                  1 = they integrate its ODE limit g = 0.
 *   "wrap"         Kuramoto phases (saved states and checkpoints):
 *                  1 (default) = every kernel returns them reduced to
 *                  [-pi, pi] (the domain of Sec. 2.2.1); the one-orbit-per-
 *                  lane kernel reduces its state after every step as the
 *                  16-lane kernels do, so a saved state resumes exactly;
 *                  0 = continuous phases, never reduced: only the
 *                  one-orbit-per-lane kernel provides them, so "kernel" auto
 *                  selects it, "kernel" 2 and sode_forward_ckpt /
 *                  sode_adjoint give SODE_EUNSUPPORTED.  Other models
 *                  ignore the option.
 *   "noise_waves"  coupled Kuramoto kernels (binary64: four lanes per orbit
 *                  for n <= 4, 16-lane rows for n <= 32 and 49 <= n <= 64;
 *                  binary32: 16-lane rows for n <= 32 and 49 <= n <= 64):
 *                  0 = every lane draws its own normals; 1 or 2 = each
 *                  workgroup is one integrating wave (16 quads or 4 rows)
 *                  and that many waves drawing their normals a batch of
 *                  steps ahead into LDS, which shortens the integrating
 *                  wave's per-step work when the ensemble is too small to
 *                  fill the chip; -1 (default) = 2 while there are at most
 *                  two integrating waves per compute unit, 1 while there
 *                  are at most four, else 0.  The normals, and so the
 *                  results, are bitwise the same in every case.  Other
 *                  kernels and row sizes ignore the option.
 *   "observable"   0 = state (q = n values per save);
 *                  1 = Kuramoto order parameter r of Eq. (7), Sec. 2.3.1
 *                      (q = 1; Kuramoto only).
 *   "kernel"       0 = auto; 1 = plain (one orbit per lane, any model,
 *                  either precision); 2 = coupled (Kuramoto, method EM,
 *                  n <= 128 in binary32, n <= 64 in binary64: 16 lanes per
 *                  orbit exchange phases
 *                  through DPP row rotations; an n that is not a multiple
 *                  of 16 runs padded with oscillators frozen at phase 0
 *                  whose coupling is cancelled; binary64 with n <= 4 uses
 *                  4 lanes per orbit and DPP quad permutations instead);
 *                  3 = matrix (see "gemm").
 *                  Auto takes coupled for binary32 Kuramoto EM with
 *                  n <= 128 (n <= 4: up to 56,000 / 120,000 / 200,000 /
 *                  110,000 orbits for n = 1..4 on 256 compute units,
 *                  scaled with the device's) and for
 *                  binary64 Kuramoto EM with n <= 64 (n = 5: up to 100,000
 *                  orbits pairwise or 60,000 mean-field, beyond which one
 *                  orbit per lane is faster),
 *                  matrix for a supported dense network, else plain.
 *   "shared_params" 0 = p is [orbits][d] (default); 1 = p is one row [d]
 *                  used by every orbit.
 *   "gemm"         matrix kernel (model "rnn", precision 32, method EM,
 *                  shared_params 1, n in {64, 128, 256}): the drift product
 *                  W tanh(X) on the matrix cores as 0 = one bfloat16
 *                  product, 1 = bfloat16 split into hi + lo with the three
 *                  products hi.hi + hi.lo + lo.hi (default), 2 = binary32
 *                  products; accumulation is binary32 in every case.
 *   "drift"        Kuramoto coupling sum: 0 = pairwise sines as in Fig. 5
 *                  (default); 1 = the exactly equivalent mean-field form
 *                  cos(theta_i) sum_j sin(theta_j) - sin(theta_i) sum_j
 *                  cos(theta_j), O(n) per orbit-step (all Kuramoto paths).
 *   "compensated"  binary32 Kuramoto kernels (coupled, forward_ckpt,
 *                  adjoint) and the ragged FHN kernel: 1 (default) carries
 *                  each state variable as hi + lo and adds every increment
 *                  with Dekker's Fast2Sum (exact while |hi| is at least the
 *                  increment, i.e. away from zero), so rounding no longer
 *                  accumulates over the steps (saved states hold hi;
 *                  resuming from them restarts lo at 0); 0 keeps a single
 *                  binary32 value (saved states resume bit-exactly).
 * Unknown keys or values give SODE_EINVAL and leave the handle unchanged.
 */
int sode_set_option(sode_t h, const char* key, int64_t value);
int sode_get_option(sode_t h, const char* key, int64_t* value);

/*
 * sode_integrate - integrate `orbits` orbits for `nsteps` steps of size dt
 * from time t0 and save the observable every `stride` steps.
 *
 *   X0   [orbits][n]            initial states X^0 (Sec. 2.1.1, re-indexed
 *                               from 0: X^0 = X0 at t0).
 *   p    [orbits][d] or [d]     parameters (see "shared_params").
 *   out  [orbits][nsave][q]     nsave = nsteps/stride + 1; out[o][s] is the
 *                               observable of X^{s*stride}, so out[o][0] is
 *                               the observable of X0.  Kuramoto phases
 *                               follow the "wrap" option whichever kernel
 *                               runs the call.
 *   nsteps >= 0, stride >= 1, nsteps % stride == 0, else SODE_EINVAL.
 *   seed  key of the Philox-4x32-10 noise stream (Sec. 2.1.2 names the
 *         Random123 family).  Normal j of orbit o at step k comes from the
 *         block with counter (k, o, j/4, 0) and key (seed mod 2^32,
 *         seed >> 32), words (2h, 2h+1), h = (j/2)%2, through Eq. (3)
 *         with U1 = ((w0 >> 8) + 1) 2^-24 and U2 = (w1 >> 8) 2^-24 (cosine
 *         for even j, sine for odd j).
 * Equivalent to sode_integrate_ex with orbit_offset = step_offset = 0 and no
 * per-orbit ids or seeds.
 */
int sode_integrate(sode_t h, const void* X0, const void* p, int64_t orbits, double t0,
                   double dt, int64_t nsteps, int64_t stride, uint64_t seed, void* out,
                   void* stream);

/*
 * sode_integrate_ex - sode_integrate with explicit noise addressing, so that
 * any orbit can be replayed bit-exactly, shards of one ensemble can run in
 * separate calls, and an integration can resume where an earlier one ended.
 * The kernel of Sec. 2.1.3 (Fig. 1) takes an array of counters for the
 * counter-based generator of Sec. 2.1.2; here the counter of every normal
 * is a function of (step, orbit id, block), and these arguments choose the
 * step and orbit ids a call uses.
 *
 *   orbit_offset  orbit o uses orbit id orbit_offset + o (mod 2^32) ...
 *   orbit_ids     ... unless this device array [orbits] (uint32) is given.
 *   orbit_seeds   device array [orbits] (uint64) of per-orbit seeds, or NULL
 *                 for `seed` everywhere.
 *   step_offset   step k of this call uses Philox counter step_offset + k;
 *                 time is still t_k = t0 + k dt.  step_offset + nsteps must
 *                 not exceed 2^32, else SODE_EINVAL.
 * Resuming: calling again with X0 = last saved state, t0 = end time and
 * step_offset = steps already done continues the same noise path; with
 * "compensated" 0 (or a binary64 handle) the continuation is bit-exact.
 */
int sode_integrate_ex(sode_t h, const void* X0, const void* p, int64_t orbits, double t0,
                      double dt, int64_t nsteps, int64_t stride, uint64_t seed,
                      uint64_t orbit_offset, uint64_t step_offset, const uint32_t* orbit_ids,
                      const uint64_t* orbit_seeds, void* out, void* stream);

/*
 * sode_forward_ckpt - Euler-Maruyama integration of Kuramoto orbits that
 * keeps what a pathwise gradient needs: every `ckpt_every`-th state and the
 * window-averaged order parameter
 *     R_o = (1/W) sum_{k = win_lo .. win_hi} r(X_o^k),  W = win_hi - win_lo + 1,
 * with r of Eq. (7) (Sec. 2.3.1), accumulated in binary64.  Parameter
 * fitting over many orbits is the use the paper builds toward (Sec. 1.2).
 *
 * Handle: model "kuramoto", precision 32, method EM, wrap 1, n in
 * {16, 32, 64, 128} (else SODE_EUNSUPPORTED).  Noise addressing as
 * sode_integrate_ex with orbit ids orbit_offset + o and the single `seed`.
 * With "compensated" 1 each phase is carried as hi + lo between
 * checkpoints and lo restarts at 0 after every checkpoint, so that stepping
 * `ckpt_every` steps from ckpt[o][c] (sode_integrate_ex with step_offset
 * c * ckpt_every) gives ckpt[o][c+1] bit for bit.  Step indices k are
 * local to the call (k = 0 is X0); 0 <= win_lo <= win_hi <= nsteps,
 * nsteps % ckpt_every == 0, else SODE_EINVAL.
 *   ckpt  [orbits][nsteps/ckpt_every + 1][n] float, ckpt[o][c] = X^{c*ckpt_every}
 *   R     [orbits] double
 */
int sode_forward_ckpt(sode_t h, const void* X0, const void* p, int64_t orbits, double t0,
                      double dt, int64_t nsteps, int64_t ckpt_every, int64_t win_lo,
                      int64_t win_hi, uint64_t seed, uint64_t orbit_offset, uint64_t step_offset,
                      void* ckpt, double* R, void* stream);

/*
 * sode_adjoint - gradient of sum_o dL_dR[o] R_o with respect to p by the
 * discrete adjoint of the Euler-Maruyama map, for checkpoints written by
 * sode_forward_ckpt with the same arguments: the parameter gradients that
 * fitting a model to data over many orbits needs (the parameter-estimation
 * use of Sec. 1.2).  The noise is regenerated from the Philox counter
 * (common random numbers), segments between checkpoints are recomputed bit
 * for bit as sode_forward_ckpt stepped them (with "compensated" 1 the
 * forward pass restarts the trailing parts at 0 at every checkpoint, so a
 * checkpoint is an exact restart point), and gradients are accumulated in
 * binary64.
 *
 *   dL_dR            [orbits] double, or NULL for all ones.
 *   grad_p           [d] double, sum over orbits in a fixed order (may be
 *                    NULL if grad_p_per_orbit is given).
 *   grad_p_per_orbit [orbits][d] double, dL_dR[o] * dR_o/dp, or NULL.
 * The library keeps a device scratch area of orbits * ckpt_every * 2n floats
 * (the recomputed states of a segment and the normals of each step)
 * (plus orbits * d doubles when grad_p_per_orbit is NULL) in the handle;
 * growing it may allocate (SODE_ENOMEM on failure).
 */
int sode_adjoint(sode_t h, const void* p, int64_t orbits, double t0, double dt, int64_t nsteps,
                 int64_t ckpt_every, int64_t win_lo, int64_t win_hi, uint64_t seed,
                 uint64_t orbit_offset, uint64_t step_offset, const void* ckpt,
                 const double* dL_dR, double* grad_p, double* grad_p_per_orbit, void* stream);

/*
 * sode_integrate_ragged - integrate a batch of instances of uneven size and
 * length in one persistent launch (the paper runs one size per launch and
 * tunes the work-group size by hand, Sec. 2.2.2 and Table 4).
 *
 * Handle: model "fhn", precision 32, method EM or Milstein (the same steps
 * for this additive noise; else SODE_EUNSUPPORTED); every
 * instance has an even n with 2 <= n <= min(256, handle n), m = n/2, d = 5.
 *   inst   HOST array [count] of descriptors (read during the call only).
 *   X0, p, out  packed DEVICE arrays of x0_len, p_len, out_len floats; every
 *          instance's slices must lie inside them (else SODE_EINVAL).
 * Instance i uses the noise of sode_integrate_ex with orbit id
 * inst[i].orbit_id and seed inst[i].seed; time t_k = t0 + k dt.
 *
 * Instances are grouped by lane shape and scheduled longest first through
 * a device work queue.  Options: "waves_per_cu" and "units_per_lane"
 * (0 = chosen by the built-in autotuner on the first call for a batch
 * shape, then cached in the handle); "graph" (1 = capture the launch in a
 * HIP graph and replay it for identical calls); "persistent" (0 = one
 * block per group, no queue: bitwise the same results, for testing).  The
 * handle keeps device copies of the schedule; rebuilding them may allocate.
 */
int sode_integrate_ragged(sode_t h, const sode_instance_t* inst, int32_t count, const void* X0,
                          int64_t x0_len, const void* p, int64_t p_len, void* out,
                          int64_t out_len, double t0, double dt, void* stream);

/*
 * sode_ensemble_stats - mean and standard deviation over orbits of every
 * column of a saved-observable array, in binary64: the ensemble statistics
 * <r(t)> and sigma(r(t)) of the accuracy study (Sec. 2.3.1-2.3.2).
 *
 *   out     [orbits][cols] DEVICE array of the handle's precision (cols =
 *           nsave * q for the output of sode_integrate).
 *   mean    [cols] double;  stddev [cols] double or NULL: sample standard
 *           deviation (denominator orbits - 1; 0 when orbits < 2).
 * The reduction order is fixed (64 orbit chunks merged in order), so the
 * result is reproducible bit for bit.  Uses the handle's scratch area
 * (64 * cols * 24 bytes; growing it may allocate).  With orbits = 0 the
 * means are 0.
 */
int sode_ensemble_stats(sode_t h, const void* out, int64_t orbits, int64_t cols, double* mean,
                        double* stddev, void* stream);

/*
 * sode_ensemble_stats_noalloc - sode_ensemble_stats for callers that cannot
 * allocate device memory: code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, same kernels and the same
 * bit-for-bit result, but the partials live in a fixed device array of the
 * library (64 orbit chunks x SODE_STATS_NOALLOC_MAX_COLS columns x 24 bytes =
 * 3 MiB per GPU, held until the process ends) instead of the handle's growable
 * scratch, so the call never allocates device memory.
 *   cols > SODE_STATS_NOALLOC_MAX_COLS -> SODE_ETOOBIG (before any HIP call).
 * The first call on a device looks the array's address up on that device
 * (a failure there -> SODE_EDEVICE).  Every call on one GPU shares that GPU's
 * array: calls that may overlap on one GPU (different streams, or different
 * host threads) race and must be serialised by the caller.  Nothing in the
 * array needs clearing between calls: each call writes every partial it
 * reads.
 */
#define SODE_STATS_NOALLOC_MAX_COLS 2048
int sode_ensemble_stats_noalloc(sode_t h, const void* out, int64_t orbits, int64_t cols,
                                double* mean, double* stddev, void* stream);

/*
 * sode_sync - wait for the handle's last launch and report device errors.
 * Returns SODE_EDEVICE if the stream reported an error, else
 * SODE_ENONFINITE if any value saved by sode_integrate(_ex) or
 * sode_integrate_ragged since the previous sode_sync was NaN or infinite
 * (the kernels raise a per-device flag of the handle; this call reads and
 * clears it), else SODE_OK.  The flag (4 bytes per device) is allocated by
 * the first integrate call on a device.
 */
int sode_sync(sode_t h);

/* sode_destroy - release the handle and everything the library owns for it.
 * NULL is accepted and ignored. */
int sode_destroy(sode_t h);

/* sode_strerror - static, NUL-terminated description of a status code. */
const char* sode_strerror(int status);

/* sode_version - library version as major*10000 + minor*100 + patch. */
int sode_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SODE_H */
