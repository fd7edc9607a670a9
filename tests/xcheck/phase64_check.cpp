// Host check of the binary64 coupled kernels' elementary functions
// (paper_1908_03869_amd/csrc/phase64.hpp) against long double:
//   minus_two_ln_u24(j) for every j = 1 .. 2^24,
//   cos_sin_turn_u24(i) for every i = 0 .. 2^24 - 1,
//   sin_phase64(x) on a dense grid of [-2 pi - 1e-9, 2 pi + 1e-9] and next
//   to the multiples of pi in that range.
// Prints one line per function: "<name> <max error in ulps of the result>
// <max absolute error> <count>"; cos / sin errors are in units of 2^-53
// (half an ulp of 1), since their values cross zero.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "phase64.hpp"

static double ulp_of(long double ref)
{
    const double r = std::fabs((double)ref);
    if (r == 0.0)
        return 4.9406564584124654e-324;
    return std::nextafter(r, INFINITY) - r;
}

int main()
{
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const long double pi = 3.141592653589793238462643383279502884L;
    double worst = 0.0, worst_abs = 0.0;
    for (uint32_t j = 1; j <= (1u << 24); ++j) {
        const long double ref = -2.0L * logl((long double)j / 16777216.0L);
        const double got = sode::minus_two_ln_u24(j);
        const long double e = fabsl((long double)got - ref);
        const double u = (double)(e / (long double)ulp_of(ref));
        if (u > worst)
            worst = u;
        if ((double)e > worst_abs)
            worst_abs = (double)e;
    }
    std::printf("minus_two_ln_u24 %.4f %.4e %u\n", worst, worst_abs, 1u << 24);

    worst = 0.0;
    worst_abs = 0.0;
    for (uint32_t i = 0; i < (1u << 24); ++i) {
        const long double ang = two_pi * ((long double)i / 16777216.0L);
        double c, s;
        sode::cos_sin_turn_u24(i, c, s);
        const long double ec = fabsl((long double)c - cosl(ang));
        const long double es = fabsl((long double)s - sinl(ang));
        const double e = (double)(ec > es ? ec : es);
        if (e > worst_abs)
            worst_abs = e;
    }
    std::printf("cos_sin_turn_u24 %.4f %.4e %u\n", worst_abs / 0x1p-53, worst_abs, 1u << 24);

    worst = 0.0;
    worst_abs = 0.0;
    long count = 0;
    const long n = 20000000;
    for (long t = 0; t <= n; ++t) {
        const double x = -6.283185308 + 12.566370616 * ((double)t / (double)n);
        const long double ref = sinl((long double)x);
        const double got = sode::sin_phase64(x);
        const long double e = fabsl((long double)got - ref);
        const double u = (double)(e / (long double)ulp_of(ref));
        if (u > worst)
            worst = u;
        if ((double)e > worst_abs)
            worst_abs = (double)e;
        ++count;
    }
    for (int k = -2; k <= 2; ++k) {
        const double c = (double)(pi * (long double)k);
        double x = c;
        for (int t = 0; t < 2000; ++t) {
            x = std::nextafter(x, INFINITY);
            for (double y : {x, 2.0 * c - x}) {
                const long double ref = sinl((long double)y);
                const long double e = fabsl((long double)sode::sin_phase64(y) - ref);
                const double u = (double)(e / (long double)ulp_of(ref));
                if (u > worst)
                    worst = u;
                ++count;
            }
        }
    }
    std::printf("sin_phase64 %.4f %.4e %ld\n", worst, worst_abs, count);
    return 0;
}
