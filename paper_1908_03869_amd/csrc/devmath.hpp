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
