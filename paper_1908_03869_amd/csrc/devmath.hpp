// devmath.hpp - precision-overloaded device math for the model functors and
// the one-orbit-per-lane kernel (also compiled at run time, hence no
// includes beyond what the run-time compiler provides).
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace sode {

__device__ __forceinline__ float dev_sin(float x) { return sinf(x); }
__device__ __forceinline__ double dev_sin(double x) { return sin(x); }
__device__ __forceinline__ float dev_cos(float x) { return cosf(x); }
__device__ __forceinline__ double dev_cos(double x) { return cos(x); }
__device__ __forceinline__ float dev_tanh(float x) { return tanhf(x); }
__device__ __forceinline__ double dev_tanh(double x) { return tanh(x); }
__device__ __forceinline__ float dev_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dev_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dev_fabs(float x) { return fabsf(x); }
__device__ __forceinline__ double dev_fabs(double x) { return fabs(x); }

// A phase reduced to [-pi, pi]: x - 2 pi rint(x / 2 pi), with 2 pi taken as
// its nearest value in the precision plus the remainder.  A phase already in
// range comes back unchanged (rint gives 0); a wrapped one rounds twice.
__device__ __forceinline__ float dev_wrap_phase(float x)
{
    const float k = __builtin_rintf(x * 0.159154943091895335768883763373f);
    x = __builtin_fmaf(-k, 6.28318548202514648437500f, x);
    return __builtin_fmaf(-k, -1.74845553146951715461e-07f, x);
}
__device__ __forceinline__ double dev_wrap_phase(double x)
{
    const double k = __builtin_rint(x * 0.15915494309189535);
    x = __builtin_fma(-k, 6.28318530717958623199592693708837032318115234375, x);
    return __builtin_fma(-k, 2.4492935982947063544521318645500021e-16, x);
}

// Raise the handle's non-finite flag (when there is one) if a value about
// to be saved is NaN or infinite: one comparison per saved value, and a
// vector atomic only in the rare failing case.
__device__ __forceinline__ void note_nonfinite(int* flag, float x)
{
    if (flag && !(__builtin_fabsf(x) <= 3.40282347e38f))
        __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void note_nonfinite(int* flag, double x)
{
    if (flag && !(__builtin_fabs(x) <= 1.7976931348623157e308))
        __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sode
