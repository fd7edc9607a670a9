// implicit_fixed_f32_euler.hip - the fixed-size implicit Euler kernels in binary32
// (implicit_fixed.hpp), one translation unit per precision and method.
#include "implicit_fixed.hpp"

namespace sode {

bool launch_implicit_fixed_f32_euler(const Request& r, hipError_t* e) { return launch_implicit_fixed<float, kImplicitEuler>(r, e); }

}  // namespace sode
