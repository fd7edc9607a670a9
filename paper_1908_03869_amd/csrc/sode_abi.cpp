// sode_abi.cpp - the C ABI of libsode (declared in include/sode.h).
//
// Every entry point validates its arguments completely before it makes any
// HIP call, so argument errors are reported synchronously (and can be tested
// on a machine without a GPU).  Dispatch then picks a kernel and launches it
// asynchronously on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "ctx.hpp"


namespace {

constexpr int kVersion = 100;  // 0.1.0

// Upper bound on orbits per call: keeps every grid (16 lanes per orbit in
// the coupled kernel) below 2^32 work-items.
constexpr int64_t kMaxOrbits = int64_t(1) << 27;

struct ModelInfo {
    const char* name;
    int id;
};
constexpr ModelInfo kModels[] = {
    {"kuramoto", sode::kKuramoto}, {"ou", sode::kOU}, {"gbm", sode::kGBM},
    {"fhn", sode::kFHN},           {"rnn", sode::kRNN},
};

// Dimensions (n equations, m noises, d parameters) each model accepts.
bool dims_match(int model, int32_t n, int32_t m, int32_t d)
{
    if (n <= 0 || m <= 0 || d <= 0)
        return false;
    switch (model) {
    case sode::kKuramoto: return m == n && (int64_t)d == 2 * (int64_t)n + 1;
    case sode::kOU: return m == n && d == 3;
    case sode::kGBM: return m == n && d == 2;
    case sode::kFHN: return n % 2 == 0 && m == n / 2 && d == 5;
    case sode::kRNN: return m == n && (int64_t)d == (int64_t)n * n + n + 1;
    default: return false;
    }
}

int status_of(hipError_t e) { return e == hipSuccess ? SODE_OK : SODE_EDEVICE; }

// Make sure the handle owns at least `bytes` of device scratch.  Memory the
// previous launch on the handle may still use is released only after that
// launch has finished.
int ensure_scratch(sode_ctx* h, size_t bytes)
{
    if (bytes <= h->scratch_bytes)
        return SODE_OK;
    if (h->scratch) {
        if (h->launched && hipStreamSynchronize(h->last_stream) != hipSuccess)
            return SODE_EDEVICE;
        (void)hipFree(h->scratch);
        h->scratch = nullptr;
        h->scratch_bytes = 0;
    }
    if (hipMalloc(&h->scratch, bytes) != hipSuccess) {
        h->scratch = nullptr;
        return SODE_ENOMEM;
    }
    h->scratch_bytes = bytes;
    return SODE_OK;
}

// Shared argument checks of the checkpointed forward pass and the adjoint.
int check_adjoint_args(const sode_ctx* h, int64_t orbits, double dt, int64_t nsteps,
                       int64_t every, int64_t win_lo, int64_t win_hi, uint64_t step_offset)
{
    if (!h)
        return SODE_EINVAL;
    if (orbits < 0 || orbits > kMaxOrbits || nsteps < 1 || every < 1 || nsteps % every != 0)
        return SODE_EINVAL;
    if (win_lo < 0 || win_hi < win_lo || win_hi > nsteps)
        return SODE_EINVAL;
    if (!std::isfinite(dt) || !(dt > 0.0))
        return SODE_EINVAL;
    if (step_offset > (1ull << 32) || (uint64_t)nsteps > (1ull << 32) - step_offset)
        return SODE_EINVAL;
    if (h->model != sode::kKuramoto || h->precision != 32 || h->method != sode::kEM ||
        !h->wrap || !sode::adjoint_supports(h->n))
        return SODE_EUNSUPPORTED;
    // Checkpoints [orbits][nsteps/every + 1][n] must fit 64-bit byte offsets.
    if (orbits > 0 && nsteps / every + 1 > (INT64_MAX / 16) / orbits / h->n)
        return SODE_EINVAL;
    return SODE_OK;
}

// Largest binary32 Kuramoto ensemble (n <= 4) for which the 16-lane row, a
// padded one, beats one orbit per lane: a short row (n <= 8) costs ~n per
// orbit, while one orbit per lane takes a fixed, latency-bound time until
// the ensemble fills the chip and ~n^2 per orbit-step after.  Paper protocol
// (8000 steps) on 256 compute units, scaled with the device's: n = 1 one
// orbit per lane from 65,536 orbits on (6.7 against 7.3 ms), n = 2 from
// 131,072 (15.3 against 16.2), n = 3 at 262,144 (32.9 against 37.3), n = 4
// (a size compiled in) from 131,072 (18.1 against 20.9); from n = 5 the row
// wins at every size measured (n = 5 at 262,144 orbits 46.2 against 50.5).
int64_t coupled32_max_orbits(int n)
{
    static const int64_t kMax256[5] = {0, 56000, 120000, 200000, 110000};
    if (n >= 5)
        return INT64_MAX;
    return kMax256[n] * sode::device_compute_units() / 256;
}

// Which kernel a request goes to; SODE_EUNSUPPORTED if none can run it.
// Auto follows the paper's speed protocol as measured here.  Binary32: the
// 16-lane Kuramoto kernel up to coupled32_max_orbits(n), else one orbit per
// lane.  Binary64: four lanes per orbit for n <= 4 and the 16-lane row for
// 6 <= n <= 64 at any size; at n = 5 (a row of 11 pads) the row up to 100,000
// orbits pairwise or 60,000 mean-field, one orbit per lane beyond.  The dense network goes to the matrix
// kernel; everything else to one orbit per lane.
int choose_kernel(const sode_ctx* h, int64_t orbits, int* kernel)
{
    // RK4 and the implicit steppers integrate the ODE limit g = 0.  A model
    // with a diffusion (every built-in model; a source-text model with
    // m > 0) is refused unless the caller asks for that limit explicitly.
    const bool ode_method = h->method == sode::kRK4 || h->method == sode::kImplicitEuler ||
                            h->method == sode::kImplicitMidpoint;
    const bool has_diffusion = h->model != sode::kCustom || h->m > 0;
    if (ode_method && has_diffusion && !h->ode_limit)
        return SODE_EUNSUPPORTED;
    if (h->model == sode::kCustom) {
        // Source-text models run on the run-time compiled plain stepper.
        const bool implicit = h->method == sode::kImplicitEuler || h->method == sode::kImplicitMidpoint;
        if ((h->kernel != 0 && h->kernel != 1) || h->method == sode::kMilstein ||
            (implicit && h->n > sode::kImplicitMaxN))
            return SODE_EUNSUPPORTED;
        *kernel = 4;
        return SODE_OK;
    }
    // The 16-lane kernels wrap the phases every step: with continuous
    // phases requested (wrap = 0) only one orbit per lane applies.
    const bool coupled_ok = h->model == sode::kKuramoto && h->method == sode::kEM && h->wrap &&
                            (h->precision == 32 ? sode::coupled_supports(h->n)
                                                : sode::coupled64_supports(h->n));
    const bool matrix_ok = h->model == sode::kRNN && h->precision == 32 && h->method == sode::kEM &&
                           h->shared_params && sode::rnn_mfma_supports(h->n);
    const bool implicit = h->method == sode::kImplicitEuler || h->method == sode::kImplicitMidpoint;
    const bool plain_ok = h->n <= (implicit ? sode::kImplicitMaxN : sode::kPlainMaxN);
    if (h->kernel == 3) {
        if (!matrix_ok)
            return SODE_EUNSUPPORTED;
        *kernel = 3;
    } else if (h->kernel == 2) {
        if (!coupled_ok)
            return SODE_EUNSUPPORTED;
        *kernel = 2;
    } else if (h->kernel == 1) {
        if (!plain_ok)
            return SODE_EUNSUPPORTED;
        *kernel = 1;
    } else if (coupled_ok && h->precision == 32 && orbits <= coupled32_max_orbits(h->n)) {
        *kernel = 2;
    } else if (coupled_ok && h->precision == 64 && (h->n != 5 || orbits <= (h->drift == 1 ? 60000 : 100000))) {
        // Binary64: four lanes per orbit (n <= 4) or a 16-lane row (6 <= n
        // <= 64) beat one orbit per lane at every ensemble size measured
        // (paper protocol, up to 196,608 orbits, pairwise and mean-field).
        // At n = 5 a row is 11/16 padding and the one-orbit-per-lane kernel,
        // whose time steps with each whole wave per SIMD, is faster from
        // about 100,000 orbits on pairwise (131,072: 60.0 against 81.8 ms;
        // the short row wins at 81,920, 51.6 against 59.7) and 65,536
        // mean-field (47.7 against 55.1).
        *kernel = 2;
    } else if (matrix_ok) {
        *kernel = 3;
    } else if (plain_ok) {
        *kernel = 1;
    } else {
        return SODE_EUNSUPPORTED;
    }
    return SODE_OK;
}

}  // namespace

namespace sode {
int* nonfinite_flag(sode_ctx* h)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return nullptr;
    const auto it = h->nonfinite.find(dev);
    if (it != h->nonfinite.end())
        return it->second;
    int* f = nullptr;
    if (hipMalloc(&f, sizeof(int)) != hipSuccess)
        return nullptr;
    if (hipMemset(f, 0, sizeof(int)) != hipSuccess) {
        (void)hipFree(f);
        return nullptr;
    }
    h->nonfinite[dev] = f;
    return f;
}
}  // namespace sode

extern "C" {

int sode_version(void) { return kVersion; }

const char* sode_strerror(int status)
{
    switch (status) {
    case SODE_OK: return "success";
    case SODE_EINVAL: return "invalid argument";
    case SODE_ENOMEM: return "out of memory";
    case SODE_EDEVICE: return "HIP device or launch error";
    case SODE_EUNSUPPORTED: return "unsupported combination of model, size and options";
    case SODE_ENONFINITE: return "non-finite value in a saved state";
    case SODE_EBUILD: return "run-time compilation of the model source failed (see sode_build_log)";
    case SODE_ETOOBIG: return "request exceeds the fixed capacity of a non-allocating entry point";
    default: return "unknown status";
    }
}

int sode_create(const char* model, int32_t n, int32_t m, int32_t d, sode_t* out)
{
    if (!model || !out)
        return SODE_EINVAL;
    *out = nullptr;
    int id = -1;
    for (const ModelInfo& mi : kModels)
        if (std::strcmp(mi.name, model) == 0)
            id = mi.id;
    if (id < 0 || !dims_match(id, n, m, d))
        return SODE_EINVAL;
    sode_ctx* h = new (std::nothrow) sode_ctx;
    if (!h)
        return SODE_ENOMEM;
    h->model = id;
    h->n = n;
    h->m = m;
    h->d = d;
    *out = h;
    return SODE_OK;
}

int sode_create_custom(const char* drift_body, const char* diffusion_body, int32_t n, int32_t m,
                       int32_t d, sode_t* out)
{
    if (!out)
        return SODE_EINVAL;
    *out = nullptr;
    if (!drift_body || (m > 0 && !diffusion_body))
        return SODE_EINVAL;
    if (n < 1 || n > sode::kPlainMaxN || m < 0 || m > sode::kPlainMaxN || d < 0)
        return SODE_EINVAL;
    sode_ctx* h = new (std::nothrow) sode_ctx;
    if (!h)
        return SODE_ENOMEM;
    h->model = sode::kCustom;
    h->n = n;
    h->m = m;
    h->d = d;
    h->drift_src = drift_body;
    h->diffusion_src = (m > 0 && diffusion_body) ? diffusion_body : "";
    *out = h;
    return SODE_OK;
}

int sode_build(sode_t h)
{
    if (!h)
        return SODE_EINVAL;
    if (h->model != sode::kCustom)
        return SODE_OK;
    return sode::rtc_build(h, h->precision);
}

int sode_build_log(sode_t h, char* buf, size_t len, size_t* needed)
{
    if (!h)
        return SODE_EINVAL;
    if (needed)
        *needed = h->build_log.size() + 1;
    if (buf && len > 0) {
        const size_t k = h->build_log.size() < len - 1 ? h->build_log.size() : len - 1;
        std::memcpy(buf, h->build_log.data(), k);
        buf[k] = '\0';
    }
    return SODE_OK;
}

int sode_set_option(sode_t h, const char* key, int64_t value)
{
    if (!h || !key)
        return SODE_EINVAL;
    if (std::strcmp(key, "precision") == 0) {
        if (value != 32 && value != 64)
            return SODE_EINVAL;
        h->precision = (int)value;
    } else if (std::strcmp(key, "method") == 0) {
        if (value < sode::kEM || value > sode::kImplicitMidpoint)
            return SODE_EINVAL;
        h->method = (int)value;
    } else if (std::strcmp(key, "observable") == 0) {
        if (value != sode::kState && value != sode::kKuramotoR)
            return SODE_EINVAL;
        if (value == sode::kKuramotoR && h->model != sode::kKuramoto)
            return SODE_EINVAL;
        h->observable = (int)value;
    } else if (std::strcmp(key, "kernel") == 0) {
        if (value < 0 || value > 3)
            return SODE_EINVAL;
        h->kernel = (int)value;
    } else if (std::strcmp(key, "gemm") == 0) {
        if (value != sode::kRnnBf16 && value != sode::kRnnBf16x3 && value != sode::kRnnFp32)
            return SODE_EINVAL;
        h->gemm = (int)value;
    } else if (std::strcmp(key, "shared_params") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->shared_params = (int)value;
    } else if (std::strcmp(key, "compensated") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->compensated = (int)value;
    } else if (std::strcmp(key, "drift") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->drift = (int)value;
    } else if (std::strcmp(key, "waves_per_cu") == 0) {
        if (value < 0 || value > 32)
            return SODE_EINVAL;
        h->waves_per_cu = (int)value;
    } else if (std::strcmp(key, "units_per_lane") == 0) {
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
            return SODE_EINVAL;
        h->units_per_lane = (int)value;
    } else if (std::strcmp(key, "graph") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->graph = (int)value;
    } else if (std::strcmp(key, "persistent") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->persistent = (int)value;
    } else if (std::strcmp(key, "ode_limit") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->ode_limit = (int)value;
    } else if (std::strcmp(key, "wrap") == 0) {
        if (value != 0 && value != 1)
            return SODE_EINVAL;
        h->wrap = (int)value;
    } else if (std::strcmp(key, "noise_waves") == 0) {
        if (value < -1 || value > 2)
            return SODE_EINVAL;
        h->noise_waves = (int)value;
    } else {
        return SODE_EINVAL;
    }
    return SODE_OK;
}

int sode_get_option(sode_t h, const char* key, int64_t* value)
{
    if (!h || !key || !value)
        return SODE_EINVAL;
    if (std::strcmp(key, "precision") == 0)
        *value = h->precision;
    else if (std::strcmp(key, "method") == 0)
        *value = h->method;
    else if (std::strcmp(key, "observable") == 0)
        *value = h->observable;
    else if (std::strcmp(key, "kernel") == 0)
        *value = h->kernel;
    else if (std::strcmp(key, "gemm") == 0)
        *value = h->gemm;
    else if (std::strcmp(key, "shared_params") == 0)
        *value = h->shared_params;
    else if (std::strcmp(key, "compensated") == 0)
        *value = h->compensated;
    else if (std::strcmp(key, "drift") == 0)
        *value = h->drift;
    else if (std::strcmp(key, "waves_per_cu") == 0)
        *value = h->waves_per_cu;
    else if (std::strcmp(key, "units_per_lane") == 0)
        *value = h->units_per_lane;
    else if (std::strcmp(key, "graph") == 0)
        *value = h->graph;
    else if (std::strcmp(key, "persistent") == 0)
        *value = h->persistent;
    else if (std::strcmp(key, "ode_limit") == 0)
        *value = h->ode_limit;
    else if (std::strcmp(key, "wrap") == 0)
        *value = h->wrap;
    else if (std::strcmp(key, "noise_waves") == 0)
        *value = h->noise_waves;
    else if (std::strcmp(key, "ragged_waves_per_cu") == 0)
        *value = h->rg_last_waves;
    else if (std::strcmp(key, "ragged_units_per_lane") == 0)
        *value = h->rg_last_units;
    else
        return SODE_EINVAL;
    return SODE_OK;
}

int sode_integrate_ex(sode_t h, const void* X0, const void* p, int64_t orbits, double t0,
                      double dt, int64_t nsteps, int64_t stride, uint64_t seed,
                      uint64_t orbit_offset, uint64_t step_offset, const uint32_t* orbit_ids,
                      const uint64_t* orbit_seeds, void* out, void* stream)
{
    if (!h)
        return SODE_EINVAL;
    if (orbits < 0 || nsteps < 0 || stride < 1 || nsteps % stride != 0)
        return SODE_EINVAL;
    if (!std::isfinite(t0) || !std::isfinite(dt) || !(dt > 0.0))
        return SODE_EINVAL;
    if (step_offset > (1ull << 32) || (uint64_t)nsteps > (1ull << 32) - step_offset)
        return SODE_EINVAL;
    if (orbits > kMaxOrbits)
        return SODE_EINVAL;
    const int64_t nsave = nsteps / stride + 1;
    const int64_t q = h->observable == sode::kKuramotoR ? 1 : h->n;
    // Element count of out must fit comfortably in 64-bit byte offsets.
    if (orbits > 0 && nsave > (INT64_MAX / 16) / orbits / q)
        return SODE_EINVAL;
    int kernel = 0;
    const int choice = choose_kernel(h, orbits, &kernel);
    if (choice != SODE_OK)
        return choice;
    if (orbits == 0)
        return SODE_OK;
    if (!X0 || !p || !out)
        return SODE_EINVAL;

    sode::Request r;
    r.model = h->model;
    r.n = h->n;
    r.m = h->m;
    r.d = h->d;
    r.X0 = X0;
    r.p = p;
    r.p_per_orbit = h->shared_params ? 0 : 1;
    r.orbits = orbits;
    r.t0 = t0;
    r.dt = dt;
    r.nsteps = nsteps;
    r.stride = stride;
    r.nsave = nsave;
    r.seed = seed;
    r.orbit_offset = orbit_offset;
    r.step_offset = step_offset;
    r.orbit_ids = orbit_ids;
    r.orbit_seeds = orbit_seeds;
    r.method = h->method;
    r.observable = h->observable;
    r.compensated = h->compensated;
    r.drift = h->drift;
    r.wrap = h->model == sode::kKuramoto && h->wrap ? 1 : 0;
    r.noise_waves = h->noise_waves;
    r.out = out;
    r.stream = static_cast<hipStream_t>(stream);
    r.nonfinite = sode::nonfinite_flag(h);
    if (!r.nonfinite)
        return SODE_ENOMEM;

    if (kernel == 4)
        return sode::rtc_launch(h, r, h->precision);
    hipError_t e;
    if (kernel == 3)
        e = sode::launch_rnn_mfma_f32(r, h->gemm);
    else if (kernel == 2)
        e = h->precision == 64 ? sode::launch_kuramoto_coupled_f64(r) : sode::launch_kuramoto_coupled_f32(r);
    else if (h->precision == 64)
        e = sode::launch_plain_f64(r);
    else
        e = sode::launch_plain_f32(r);
    h->last_error = e;
    h->last_stream = r.stream;
    h->launched = true;
    return status_of(e);
}

int sode_integrate(sode_t h, const void* X0, const void* p, int64_t orbits, double t0,
                   double dt, int64_t nsteps, int64_t stride, uint64_t seed, void* out,
                   void* stream)
{
    return sode_integrate_ex(h, X0, p, orbits, t0, dt, nsteps, stride, seed, 0, 0, nullptr,
                             nullptr, out, stream);
}

int sode_sync(sode_t h)
{
    if (!h)
        return SODE_EINVAL;
    if (!h->launched)
        return SODE_OK;
    const hipError_t e = hipStreamSynchronize(h->last_stream);
    if (e != hipSuccess)
        return SODE_EDEVICE;
    const int st = status_of(h->last_error);
    if (st != SODE_OK)
        return st;
    for (auto& kv : h->nonfinite) {
        int v = 0;
        if (hipMemcpy(&v, kv.second, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            return SODE_EDEVICE;
        if (v) {
            if (hipMemset(kv.second, 0, sizeof(int)) != hipSuccess)
                return SODE_EDEVICE;
            return SODE_ENONFINITE;
        }
    }
    return SODE_OK;
}

int sode_forward_ckpt(sode_t h, const void* X0, const void* p, int64_t orbits, double t0,
                      double dt, int64_t nsteps, int64_t ckpt_every, int64_t win_lo,
                      int64_t win_hi, uint64_t seed, uint64_t orbit_offset, uint64_t step_offset,
                      void* ckpt, double* R, void* stream)
{
    const int st = check_adjoint_args(h, orbits, dt, nsteps, ckpt_every, win_lo, win_hi, step_offset);
    if (st != SODE_OK)
        return st;
    if (!std::isfinite(t0))
        return SODE_EINVAL;
    if (orbits == 0)
        return SODE_OK;
    if (!X0 || !p || !ckpt || !R)
        return SODE_EINVAL;
    sode::AdjointRequest r{};
    r.n = h->n;
    r.X0 = X0;
    r.p = p;
    r.p_per_orbit = h->shared_params ? 0 : 1;
    r.compensated = h->compensated;
    r.drift = h->drift;
    r.orbits = orbits;
    r.dt = dt;
    r.nsteps = nsteps;
    r.every = ckpt_every;
    r.win_lo = win_lo;
    r.win_hi = win_hi;
    r.seed = seed;
    r.orbit_offset = orbit_offset;
    r.step_offset = step_offset;
    r.ckpt = ckpt;
    r.R = R;
    r.stream = static_cast<hipStream_t>(stream);
    const hipError_t e = sode::launch_kuramoto_forward_ckpt_f32(r);
    h->last_error = e;
    h->last_stream = r.stream;
    h->launched = true;
    return status_of(e);
}

int sode_adjoint(sode_t h, const void* p, int64_t orbits, double t0, double dt, int64_t nsteps,
                 int64_t ckpt_every, int64_t win_lo, int64_t win_hi, uint64_t seed,
                 uint64_t orbit_offset, uint64_t step_offset, const void* ckpt,
                 const double* dL_dR, double* grad_p, double* grad_p_per_orbit, void* stream)
{
    const int st = check_adjoint_args(h, orbits, dt, nsteps, ckpt_every, win_lo, win_hi, step_offset);
    if (st != SODE_OK)
        return st;
    if (!std::isfinite(t0))
        return SODE_EINVAL;
    if (!grad_p && !grad_p_per_orbit)
        return SODE_EINVAL;
    if (orbits > 0 && (!p || !ckpt))
        return SODE_EINVAL;
    const size_t d = 2 * (size_t)h->n + 1;
    // Segment states and normals: [orbits][ckpt_every][2 n] floats.
    const size_t seg_bytes = (size_t)orbits * (size_t)ckpt_every * (size_t)h->n * 2 * sizeof(float);
    const size_t rows_bytes = grad_p_per_orbit ? 0 : (size_t)orbits * d * sizeof(double);
    const size_t rows_offset = (seg_bytes + 255) / 256 * 256;
    const int sc = ensure_scratch(h, rows_offset + rows_bytes + 256);
    if (sc != SODE_OK)
        return sc;
    sode::AdjointRequest r{};
    r.n = h->n;
    r.p = p;
    r.p_per_orbit = h->shared_params ? 0 : 1;
    r.compensated = h->compensated;
    r.drift = h->drift;
    r.orbits = orbits;
    r.dt = dt;
    r.nsteps = nsteps;
    r.every = ckpt_every;
    r.win_lo = win_lo;
    r.win_hi = win_hi;
    r.seed = seed;
    r.orbit_offset = orbit_offset;
    r.step_offset = step_offset;
    r.ckpt = const_cast<void*>(ckpt);
    r.dL_dR = dL_dR;
    r.grad = grad_p;
    r.grad_rows = grad_p_per_orbit
                      ? grad_p_per_orbit
                      : reinterpret_cast<double*>(static_cast<char*>(h->scratch) + rows_offset);
    r.seg_scratch = static_cast<float*>(h->scratch);
    r.stream = static_cast<hipStream_t>(stream);
    const hipError_t e = sode::launch_kuramoto_adjoint_f32(r);
    h->last_error = e;
    h->last_stream = r.stream;
    h->launched = true;
    return status_of(e);
}

}  // extern "C"

namespace {

// Argument checks and orbit partition shared by both statistics entry
// points.  SODE_OK with *empty set when there is nothing to compute.
int stats_request(sode_t h, const void* out, int64_t orbits, int64_t cols, double* mean,
                  double* stddev, void* stream, sode::StatsRequest* r, bool* empty)
{
    *empty = false;
    if (!h || orbits < 0 || cols < 0)
        return SODE_EINVAL;
    if (cols == 0) {
        *empty = true;
        return SODE_OK;
    }
    if (!mean || (orbits > 0 && !out))
        return SODE_EINVAL;
    if (orbits > 0 && cols > INT64_MAX / 16 / orbits)
        return SODE_EINVAL;
    if ((cols + 255) / 256 > INT32_MAX)
        return SODE_EINVAL;
    *r = sode::StatsRequest{};
    r->x = out;
    r->precision = h->precision;
    r->orbits = orbits;
    r->cols = cols;
    // About 64 orbit chunks, fewer for small ensembles.
    r->groups = orbits < sode::kStatsChunks ? (orbits > 0 ? orbits : 1) : sode::kStatsChunks;
    r->chunk = orbits > 0 ? (orbits + r->groups - 1) / r->groups : 1;
    r->groups = orbits > 0 ? (orbits + r->chunk - 1) / r->chunk : 1;
    r->mean = mean;
    r->stddev = stddev;
    r->stream = static_cast<hipStream_t>(stream);
    return SODE_OK;
}

int stats_launch(sode_t h, const sode::StatsRequest& r)
{
    const hipError_t e = sode::launch_ensemble_stats(r);
    h->last_error = e;
    h->last_stream = r.stream;
    h->launched = true;
    return status_of(e);
}

}  // namespace

extern "C" {

int sode_ensemble_stats(sode_t h, const void* out, int64_t orbits, int64_t cols, double* mean,
                        double* stddev, void* stream)
{
    sode::StatsRequest r;
    bool empty = false;
    const int st = stats_request(h, out, orbits, cols, mean, stddev, stream, &r, &empty);
    if (st != SODE_OK || empty)
        return st;
    const size_t need = (size_t)r.groups * (size_t)cols * sode::stats_partial_bytes();
    const int sc = ensure_scratch(h, need);
    if (sc != SODE_OK)
        return sc;
    r.scratch = h->scratch;
    return stats_launch(h, r);
}

int sode_ensemble_stats_noalloc(sode_t h, const void* out, int64_t orbits, int64_t cols,
                                double* mean, double* stddev, void* stream)
{
    sode::StatsRequest r;
    bool empty = false;
    const int st = stats_request(h, out, orbits, cols, mean, stddev, stream, &r, &empty);
    if (st != SODE_OK || empty)
        return st;
    if (cols > SODE_STATS_NOALLOC_MAX_COLS)
        return SODE_ETOOBIG;
    hipError_t e = hipSuccess;
    r.scratch = sode::stats_static_scratch(&e);
    if (!r.scratch) {
        h->last_error = e;
        return SODE_EDEVICE;
    }
    return stats_launch(h, r);
}

int sode_destroy(sode_t h)
{
    if (!h)
        return SODE_OK;
    if (h->launched)
        (void)hipStreamSynchronize(h->last_stream);
    if (h->scratch)
        (void)hipFree(h->scratch);
    sode::release_ragged(h);
    sode::rtc_release(h);
    for (auto& kv : h->nonfinite)
        (void)hipFree(kv.second);
    delete h;
    return SODE_OK;
}

}  // extern "C"
