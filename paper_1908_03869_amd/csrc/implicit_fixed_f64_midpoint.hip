// implicit_fixed_f64_midpoint.hip - the fixed-size implicit midpoint kernels in binary64
// (implicit_fixed.hpp), one translation unit per precision and method.
#include "implicit_fixed.hpp"

namespace sode {

bool launch_implicit_fixed_f64_midpoint(const Request& r, hipError_t* e) { return launch_implicit_fixed<double, kImplicitMidpoint>(r, e); }

}  // namespace sode
