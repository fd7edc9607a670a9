// launch.hpp - interface between the C ABI layer and the kernel launchers.
// Everything here is internal to libsode; arguments have been validated by
// the ABI layer before any launcher is called.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kinds.hpp"
#include "sode.h"

namespace sode {

// Compute units of the current device (256 if the query fails).
inline int device_compute_units()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

// One integrate request, already checked for shape and range.
struct Request {
    int model;
    int n, m, d;
    const void* X0;  // [orbits][n]
    const void* p;   // [orbits][d] or [d]
    int p_per_orbit; // 1: row o of p belongs to orbit o; 0: one shared row
    int64_t orbits;
    double t0, dt;
    int64_t nsteps, stride, nsave;
    uint64_t seed, orbit_offset, step_offset;
    const uint32_t* orbit_ids;    // device, may be null
    const uint64_t* orbit_seeds;  // device, may be null
    int method;
    int observable;
    int compensated;  // binary32 coupled kernels: state carried as hi + lo (Fast2Sum)
    int drift;        // Kuramoto coupling sum: 0 pairwise, 1 mean-field identity
    int wrap;         // Kuramoto: phases reduced to [-pi, pi] (the coupled kernels always do)
    int noise_waves;  // binary64 four-lane Kuramoto: waves drawing normals per integrating wave, -1 auto
    void* out;  // [orbits][nsave][q]
    int* nonfinite;  // device flag raised by a NaN or infinite save (may be null)
    hipStream_t stream;
};

// Largest state dimension of the one-orbit-per-lane kernel.
constexpr int kPlainMaxN = 128;

// Kernel arguments of the one-orbit-per-lane stepper (plain_kernel.hpp),
// filled from a request (plain.hip).
template <typename R>
struct PlainArgs;
template <typename R>
PlainArgs<R> plain_args(const Request& r);

// One orbit per lane, any model, binary64 or binary32 (the paper's design:
// one work-item per orbit).  Returns a hipError_t.
hipError_t launch_plain_f64(const Request& r);
hipError_t launch_plain_f32(const Request& r);
// Explicit steppers with a compile-time state size (plain_fixed.hip): true if
// one exists for the request's model and n (its launch status in *e).
bool launch_plain_fixed_f64(const Request& r, hipError_t* e);
bool launch_plain_fixed_f32(const Request& r, hipError_t* e);
// Implicit Euler / implicit midpoint on the ODE limit, n <= kImplicitMaxN
// (plain_implicit.hip; reached through the two launchers above).
hipError_t launch_plain_implicit_f64(const Request& r);
// Fixed-size implicit kernels (n = 1, 2, 3, 4, 6, 8): true if one took the
// request, its launch status in *e.
bool launch_implicit_fixed_f64_euler(const Request& r, hipError_t* e);
bool launch_implicit_fixed_f64_midpoint(const Request& r, hipError_t* e);
bool launch_implicit_fixed_f32_euler(const Request& r, hipError_t* e);
bool launch_implicit_fixed_f32_midpoint(const Request& r, hipError_t* e);
hipError_t launch_plain_implicit_f32(const Request& r);

// Kuramoto, binary32, Euler-Maruyama: 16 lanes per orbit, any n <= 128
// (sizes that are not multiples of 16 run padded).  The checkpointed forward
// pass and the adjoint take n in {16, 32, 64, 128}.
bool coupled_supports(int n);
bool adjoint_supports(int n);
hipError_t launch_kuramoto_coupled_f32(const Request& r);
// The same mapping in binary64 (kuramoto_coupled64.hip), n <= 64.
bool coupled64_supports(int n);
hipError_t launch_kuramoto_coupled_f64(const Request& r);

// Checkpointed forward pass and adjoint of the window-averaged order
// parameter (Kuramoto, binary32, same sizes as the coupled kernel).
struct AdjointRequest {
    int n;
    const void* X0;        // forward: [orbits][n]
    const void* p;         // [orbits][d] or [d]
    int p_per_orbit;
    int compensated;
    int drift;
    int64_t orbits;
    double dt;
    int64_t nsteps, every, win_lo, win_hi;
    uint64_t seed, orbit_offset, step_offset;
    void* ckpt;            // [orbits][nsteps/every + 1][n]
    double* R;             // forward: [orbits]
    const double* dL_dR;   // adjoint: [orbits] or null (ones)
    double* grad;          // adjoint: [d] or null
    double* grad_rows;     // adjoint: [orbits][d] per-orbit rows (caller's or scratch)
    float* seg_scratch;    // adjoint: [orbits][every][n]
    hipStream_t stream;
};
hipError_t launch_kuramoto_forward_ckpt_f32(const AdjointRequest& r);
hipError_t launch_kuramoto_adjoint_f32(const AdjointRequest& r);

// Ensemble statistics over orbits of a saved-observable array (binary64).
struct StatsRequest {
    const void* x;   // [orbits][cols] of the given precision
    int precision;   // 32 or 64
    int64_t orbits, cols;
    int64_t groups, chunk;  // orbit chunks of the first pass
    void* scratch;          // groups * cols partials
    double* mean;           // [cols]
    double* stddev;         // [cols] or null
    hipStream_t stream;
};
size_t stats_partial_bytes();
hipError_t launch_ensemble_stats(const StatsRequest& r);
// The non-allocating variant's fixed device scratch: kStatsStaticPartials
// partials (64 orbit chunks x SODE_STATS_NOALLOC_MAX_COLS columns).  Returns
// the current device's address of it (looked up once per device), or
// nullptr with *err set.
constexpr int64_t kStatsChunks = 64;
constexpr int64_t kStatsStaticPartials = kStatsChunks * SODE_STATS_NOALLOC_MAX_COLS;
void* stats_static_scratch(hipError_t* err);

// Dense random networks with the drift's matrix product on MFMA (binary32
// state, shared parameters, n in {64, 128, 256}).
enum RnnGemm : int { kRnnBf16 = 0, kRnnBf16x3 = 1, kRnnFp32 = 2 };
bool rnn_mfma_supports(int n);
hipError_t launch_rnn_mfma_f32(const Request& r, int mode);

// Ragged FitzHugh-Nagumo batches (binary32).  A group is up to
// kRaggedSlots instances of one lane shape (L lanes x U units per lane).
constexpr int kRaggedSlots = 16;
constexpr int kRaggedShapes = 20;  // L in {4, 8, 16, 32, 64} x U in {1, 2, 4, 8}
struct RaggedKernelArgs {
    const sode_instance_t* desc;  // device copy of the descriptors
    const int32_t* slots;         // [ngroups][kRaggedSlots] instance index or -1
    const int32_t* shape;         // [ngroups] shape code (ragged_shape_code) | issue priority << 8
    uint32_t* counter;            // queue ticket counter
    int32_t ngroups;
    const float* X0;
    const float* p;
    float* out;
    float dt, sqdt;
    int compensated;  // v and w carried as hi + lo (Fast2Sum)
    int* nonfinite;   // device flag raised by a NaN or infinite save (may be null)
};
int ragged_shape_code(int lanes, int units);
hipError_t launch_fhn_ragged(const RaggedKernelArgs& a, int persistent, int waves, hipStream_t stream);

}  // namespace sode
