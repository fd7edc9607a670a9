// kinds.hpp - integer codes shared by the ABI layer, the launchers and the
// kernels (also compiled at run time for models given as source text, so
// this header includes nothing).
#pragma once

namespace sode {

enum ModelId : int { kKuramoto = 0, kOU = 1, kGBM = 2, kFHN = 3, kRNN = 4, kCustom = 5 };
enum MethodId : int {
    kEM = 0,
    kRK4 = 1,
    kMilstein = 2,
    kImplicitEuler = 3,
    kImplicitMidpoint = 4
};
enum ObservableId : int { kState = 0, kKuramotoR = 1 };

// Largest state dimension of the implicit ODE steppers (each lane holds an
// n x n Newton matrix).
constexpr int kImplicitMaxN = 16;

}  // namespace sode
