// phase64.hpp - binary64 elementary functions of the binary64 coupled
// Kuramoto kernels, for the arguments those kernels produce: the sine of a
// phase or of a difference of two phases, and the Box-Muller pair of two
// 24-bit uniforms.  Host and device: a CPU test checks them against long
// double on every input the Box-Muller pair can receive, and the op-rate
// microbenchmark measures their issue cost.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace sode {

namespace phase64 {
constexpr double kPiHi = 3.1415926535897931160;        // binary64 nearest to pi
constexpr double kPiLo = 1.2246467991473531772e-16;    // pi - kPiHi
constexpr double kInvPi = 0.31830988618379067154;      // binary64 nearest to 1/pi
constexpr double kTwoPi = 6.283185307179586;           // binary64 nearest to 2 pi
// ln 2 = kLn2Hi + kLn2Lo, kLn2Hi with 29 significant bits, so that k kLn2Hi
// is exact for integers |k| < 2^24.
constexpr double kLn2Hi = 0.6931471806019545;
constexpr double kLn2Lo = -4.2009150726810846e-11;
constexpr double kSqrtHalf = 0.70710678118654752440;
}  // namespace phase64

// sin(x) for the kernels' arguments, differences of wrapped phases and the
// phases themselves (|x| <= 2 pi plus a few ulp; accurate for |x| up to
// about 2^20).  x = k pi + r with k = rint(x / pi), |r| <= pi/2, pi taken as
// two binary64 parts (Cody and Waite's reduction: the first product is exact
// for these k, so r is within an ulp); sin(x) = (-1)^k sin(r), the sign put
// on r since sin is odd; sin(r) = r + r^3 q(r^2) with q of degree 7, the
// polynomial interpolating (sin r - r) / r^3 at the 8 Chebyshev nodes of
// [0, (pi/2)^2] (phase64_coefficients.py computes it exactly from the
// Maclaurin series): relative error below 4e-17 before rounding, with two
// multiply-adds fewer than the Maclaurin series through r^21 that it
// replaces.  Within 2 ulp (largest near pi/2, from the last rounding of
// r + r^3 q).  Compiled: 13 binary64 multiplies and FMAs, a rounding, a
// conversion and two 32-bit operations, where the device library's sin
// spends about sixty binary64 issue slots on a reduction built for any
// argument.  NaN and infinities give NaN.
__host__ __device__ __forceinline__ double sin_phase64(double x)
{
    const double k = rint(x * phase64::kInvPi);
    double r = fma(-k, phase64::kPiHi, x);
    r = fma(-k, phase64::kPiLo, r);
    const uint64_t odd = (uint64_t)((int)k & 1) << 63;
    r = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, r) ^ odd);
    const double r2 = r * r;
    double q = 2.7314447669863995e-15;
    q = fma(q, r2, -7.643970296798572e-13);
    q = fma(q, r2, 1.6058977312464087e-10);
    q = fma(q, r2, -2.5052107616996182e-08);
    q = fma(q, r2, 2.7557319219163234e-06);
    q = fma(q, r2, -0.00019841269841254974);
    q = fma(q, r2, 0.008333333333333316);
    q = fma(q, r2, -0.16666666666666666);
    return fma(r * r2, q, r);
}

// -2 ln(U1) for U1 = j 2^-24, j = 1 .. 2^24 (the Box-Muller uniform of
// Eq. (3) as the counter words give it).  j = 2^e m with m in [sqrt(1/2),
// sqrt(2)), read from the bits of (double)j; then -2 ln U1 = 2 (24 - e) ln 2
// - 2 ln m, with ln m = 2 atanh(f), f = (m - 1) / (m + 1), |f| <= 0.1716,
// from the series f + f^3/3 + ... through f^21 (the rest is below
// f^22 / 23 = 6e-19 relative to f).  The integer part takes ln 2 in two
// pieces, so it is exact before the last rounding.  Within 2 ulp.
__host__ __device__ __forceinline__ double minus_two_ln_u24(uint32_t j)
{
    const uint64_t bits = __builtin_bit_cast(uint64_t, (double)j);
    int e = (int)(bits >> 52) - 1023;
    double m = __builtin_bit_cast(double, (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > 2.0 * phase64::kSqrtHalf) {  // m in (sqrt 2, 2): halve it, exactly
        m *= 0.5;
        ++e;
    }
    // j has at most 24 significant bits, so m - 1 and m + 1 are exact.
    const double f = (m - 1.0) / (m + 1.0);
    const double s = f * f;
    double p = 0.047619047619047616;  // 1/21
    p = fma(p, s, 0.05263157894736842);   // 1/19
    p = fma(p, s, 0.058823529411764705);  // 1/17
    p = fma(p, s, 0.06666666666666667);   // 1/15
    p = fma(p, s, 0.07692307692307693);   // 1/13
    p = fma(p, s, 0.09090909090909091);   // 1/11
    p = fma(p, s, 0.1111111111111111);    // 1/9
    p = fma(p, s, 0.14285714285714285);   // 1/7
    p = fma(p, s, 0.2);                   // 1/5
    p = fma(p, s, 0.3333333333333333);    // 1/3
    const double t = -4.0 * f;            // -2 ln m = -4 atanh f
    const double neg_two_ln_m = fma(t * s, p, t);
    const double k2 = (double)(2 * (24 - e));
    return fma(k2, phase64::kLn2Hi, fma(k2, phase64::kLn2Lo, neg_two_ln_m));
}

// cos(2 pi U2) and sin(2 pi U2) for U2 = i 2^-24, i = 0 .. 2^24 - 1.  The
// quarter turn q = rint(4 U2) and the rest r = U2 - q/4 (|r| <= 1/8) are
// exact; a = 2 pi r (one rounding, |a| <= pi/4) goes through the Maclaurin
// series of sin through a^17 and of cos through a^18 (truncation below
// 1e-19), and the quarter turn permutes and negates the two.  Within 2 ulp.
__host__ __device__ __forceinline__ void cos_sin_turn_u24(uint32_t i, double& c_out, double& s_out)
{
    const double u = (double)i * 0x1p-24;
    const double q = rint(4.0 * u);
    const double r = fma(q, -0.25, u);
    const double a = r * phase64::kTwoPi;
    const double a2 = a * a;
    double ps = 2.8114572543455206e-15;   //  1/17!
    ps = fma(ps, a2, -7.647163731819816e-13);   // -1/15!
    ps = fma(ps, a2, 1.6059043836821613e-10);   //  1/13!
    ps = fma(ps, a2, -2.505210838544172e-08);   // -1/11!
    ps = fma(ps, a2, 2.7557319223985893e-06);   //  1/9!
    ps = fma(ps, a2, -0.0001984126984126984);   // -1/7!
    ps = fma(ps, a2, 0.008333333333333333);     //  1/5!
    ps = fma(ps, a2, -0.16666666666666666);     // -1/3!
    const double sn = fma(a * a2, ps, a);
    double pc = -1.5619206968586225e-16;  // -1/18!
    pc = fma(pc, a2, 4.779477332387385e-14);    //  1/16!
    pc = fma(pc, a2, -1.1470745597729725e-11);  // -1/14!
    pc = fma(pc, a2, 2.08767569878681e-09);     //  1/12!
    pc = fma(pc, a2, -2.755731922398589e-07);   // -1/10!
    pc = fma(pc, a2, 2.48015873015873e-05);     //  1/8!
    pc = fma(pc, a2, -0.001388888888888889);    // -1/6!
    pc = fma(pc, a2, 0.041666666666666664);     //  1/4!
    const double cs = fma(a2, fma(a2, pc, -0.5), 1.0);
    // angle = q pi/2 + a: (cos, sin) = (c, s), (-s, c), (-c, -s), (s, -c).
    const int qi = (int)q & 3;
    const double cc = (qi & 1) ? sn : cs;
    const double ss = (qi & 1) ? cs : sn;
    c_out = ((qi + 1) & 2) ? -cc : cc;
    s_out = (qi & 2) ? -ss : ss;
}

// Box-Muller pair of Eq. (3) from two Philox words, the same uniforms and
// order as box_muller_f64 (noise.hpp): U1 = ((a >> 8) + 1) 2^-24 in (0, 1],
// U2 = (b >> 8) 2^-24 in [0, 1), z_cos = sqrt(-2 ln U1) cos(2 pi U2) first.
// The logarithm and the cosine / sine are the functions above, which use
// that the uniforms are 24-bit; the square root is the device library's.
// Within a few ulp of the library-function pair (a CPU test checks every
// possible U1 and U2).
__host__ __device__ __forceinline__ void box_muller_f64_u24(uint32_t a, uint32_t b, double& z_cos,
                                                            double& z_sin)
{
    const double radius = sqrt(minus_two_ln_u24((a >> 8) + 1u));
    double c, s;
    cos_sin_turn_u24(b >> 8, c, s);
    z_cos = radius * c;
    z_sin = radius * s;
}

}  // namespace sode
