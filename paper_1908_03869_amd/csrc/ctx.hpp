// ctx.hpp - the handle behind sode_t (internal to libsode).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>

#include "launch.hpp"

namespace sode {
struct RtcState;
}

struct sode_ctx {
    int model;
    int32_t n, m, d;
    int precision = 32;
    int method = sode::kEM;
    int observable = sode::kState;
    int kernel = 0;  // 0 auto, 1 plain, 2 coupled, 3 matrix (dense network)
    int shared_params = 0;
    int compensated = 1;
    int drift = 0;  // Kuramoto coupling: 0 pairwise sines, 1 mean-field identity
    int gemm = sode::kRnnBf16x3;  // dense-network matrix product variant
    // ODE methods (RK4, implicit) on a model with a diffusion: 0 = refused,
    // 1 = integrate the ODE limit g = 0.
    int ode_limit = 0;
    // Kuramoto phases: 1 = every kernel returns them reduced to [-pi, pi];
    // 0 = continuous phases (one-orbit-per-lane kernel only).
    int wrap = 1;
    // Binary64 four-lane Kuramoto form: waves drawing the normals per
    // integrating wave (0, 1 or 2); -1 = by ensemble size.
    int noise_waves = -1;
    // Ragged batches: 0 = autotuned.
    int waves_per_cu = 0;
    int units_per_lane = 0;
    int graph = 1;
    int persistent = 1;

    hipError_t last_error = hipSuccess;
    hipStream_t last_stream = nullptr;
    bool launched = false;

    // Device scratch of the adjoint (segment states, per-orbit rows).
    void* scratch = nullptr;
    size_t scratch_bytes = 0;

    // Device copy of the current ragged schedule:
    // [descriptors | group slots | group shapes | queue counter].
    void* rg_buf = nullptr;
    size_t rg_bytes = 0;
    size_t rg_slots_off = 0, rg_shape_off = 0, rg_counter_off = 0;
    uint64_t rg_plan_key = 0;
    int32_t rg_ngroups = 0;
    // Autotuner results, keyed by the batch shape: (waves per CU, units).
    std::map<uint64_t, std::pair<int, int>> rg_tuned;
    int rg_last_waves = 0, rg_last_units = 0;
    // Captured launch and the call it belongs to.
    hipGraph_t rg_graph = nullptr;
    hipGraphExec_t rg_exec = nullptr;
    uint64_t rg_graph_key = 0;
    hipStream_t rg_capture = nullptr;

    // Per device: a flag the kernels raise when a saved value is NaN or
    // infinite; read and cleared by sode_sync.
    std::map<int, int*> nonfinite;

    // Model given as source text (model == kCustom): the two function
    // bodies, the compiled code objects and loaded modules, the last log.
    std::string drift_src, diffusion_src, build_log;
    sode::RtcState* rtc = nullptr;
};

namespace sode {
void release_ragged(sode_ctx* h);
// The non-finite flag of the current device (allocated and cleared on first
// use); null if that fails.
int* nonfinite_flag(sode_ctx* h);
// Compile the handle's source-text model for a precision (no device needed).
int rtc_build(sode_ctx* h, int precision);
// Compile if needed, load on the current device and launch.
int rtc_launch(sode_ctx* h, const Request& r, int precision);
void rtc_release(sode_ctx* h);
}
