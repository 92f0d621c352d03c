// Accuracy check of pf::sincos_rad (host compilation of the kernel source)
// against the x87 80-bit sinl/cosl, and the kernels' shortcut for quadrant
// count 0: sincos_series(x) must give sincos_rad(x)'s bits.  Prints:
// max absolute error, max error in ulps where |result| >= 2^-10, the number
// of samples, the number of quadrant-0 samples and how many of them differ
// in any bit.
#include "../../paper_2302_10736_amd/csrc/pf_math.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

int main() {
    std::mt19937_64 rng(2302);
    long double max_abs = 0, max_ulp = 0;
    long n = 0, n0 = 0, n0_diff = 0;
    auto check = [&](double x) {
        double s, c;
        pf::sincos_rad(x, &s, &c, pf::kSinCosTaylor);
        if (pf::sincos_quadrant(x) == 0.0) {
            double s0, c0;
            pf::sincos_series(x, &s0, &c0, pf::kSinCosTaylor);
            ++n0;
            if (std::memcmp(&s, &s0, sizeof s) != 0 || std::memcmp(&c, &c0, sizeof c) != 0) ++n0_diff;
        }
        const long double rs = sinl((long double)x), rc = cosl((long double)x);
        for (int k = 0; k < 2; ++k) {
            const long double ref = k ? rc : rs;
            const double got = k ? c : s;
            const long double e = fabsl((long double)got - ref);
            if (e > max_abs) max_abs = e;
            if (fabsl(ref) >= 1.0L / 1024) {
                const long double ulp = ldexpl(1.0L, ilogbl(ref) - 52);
                if (e / ulp > max_ulp) max_ulp = e / ulp;
            }
        }
        ++n;
    };
    const double spans[] = {1e-300, 1e-8, 0.5, 0.785398, 1.0, 3.2, 10.0, 100.0, 1e3, 1e4, 1.3e5, 1e6};
    for (double a : spans) {
        std::uniform_real_distribution<double> u(-a, a);
        for (int i = 0; i < 200000; ++i) check(u(rng));
    }
    // near multiples of pi/4 and pi/2, where reduction and quadrant switch
    for (int k = -4000; k <= 4000; ++k) {
        const double base = k * 0.78539816339744830962;
        for (int d = -3; d <= 3; ++d) check(std::nextafter(base, d < 0 ? -1e300 : 1e300) + d * 1e-17);
    }
    // both sides of the quadrant-0 boundary (x * 2/pi rounding to +-0.5)
    for (double b : {0.78539816339744830962, -0.78539816339744830962})
        for (int d = -2000; d <= 2000; ++d) {
            double x = b;
            for (int q = 0; q < (d < 0 ? -d : d); ++q) x = std::nextafter(x, d < 0 ? 0.0 : 2 * b);
            check(x);
        }
    for (double x : {0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, -1e-300})
        check(x);
    printf("%.6Le %.4Lf %ld %ld %ld\n", max_abs, max_ulp, n, n0, n0_diff);
    return 0;
}
