// Double-precision sine and cosine for the evaluation kernels.
//
// Method: Cody-Waite argument reduction modulo pi/2 with a two-term split of
// pi/2 applied through fused multiply-adds, then the Taylor series of sin and
// cos on [-pi/4, pi/4]: sin through the x^17 term and cos through the x^18
// term, whose first omitted terms (x^19/19!, x^20/20!) are below 1e-19 there,
// evaluated by Horner's rule.  The quadrant (n mod 4) permutes and negates the
// two results.  Arguments with |x| >= 2^17 (or non-finite) take the runtime's
// sin and cos instead; angle differences in power-flow states never come near
// that bound.
//
// The function is plain C++ usable from host and device code, so its accuracy
// is tested on the CPU with the same source.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

namespace pf {

// Series coefficients, highest degree first: sin(r) = r + r z S(z) and
// cos(r) = 1 - z C(z) with z = r^2, S(z) = sum_k (-1)^k z^(k-1)/(2k+1)!
// (k = 1..8) and C(z) = sum_k (-1)^(k+1) z^(k-1)/(2k)! (k = 1..9).
struct SinCosCoef {
    double s[8];
    double c[9];
};

inline constexpr SinCosCoef kSinCosTaylor = {
    {2.8114572543455207632e-15,     // 1/17!
     -7.6471637318198164759e-13,    // -1/15!
     1.6059043836821614599e-10,     // 1/13!
     -2.5052108385441718775e-08,    // -1/11!
     2.7557319223985890653e-06,     // 1/9!
     -1.9841269841269841270e-04,    // -1/7!
     8.3333333333333333333e-03,     // 1/5!
     -1.6666666666666666667e-01},   // -1/3!
    {1.5619206968586225618e-16,     // 1/18!
     -4.7794773323873852974e-14,    // -1/16!
     1.1470745597729724714e-11,     // 1/14!
     -2.0876756987868098979e-09,    // -1/12!
     2.7557319223985890653e-07,     // 1/10!
     -2.4801587301587301587e-05,    // -1/8!
     1.3888888888888888889e-03,     // 1/6!
     -4.1666666666666666667e-02,    // -1/4!
     5.0000000000000000000e-01}};   // 1/2!

// Quadrant count of the reduction: x * 2/pi rounded to the nearest integer.
__host__ __device__ inline double sincos_quadrant(double x) {
    constexpr double kTwoOverPi = 0.63661977236758134308;  // 2/pi
    return rint(x * kTwoOverPi);
}

// The two series on a reduced argument r (|r| <= pi/4 + a rounding error).
__host__ __device__ inline void sincos_series(double r, double *s, double *c, const SinCosCoef &k) {
    const double z = r * r;
    double ps = k.s[0];
    for (int q = 1; q < 8; ++q) ps = fma(ps, z, k.s[q]);
    *s = fma(ps * z, r, r);
    double pc = k.c[0];
    for (int q = 1; q < 9; ++q) pc = fma(pc, z, k.c[q]);
    *c = fma(-pc, z, 1.0);
}

// `k` is kSinCosTaylor itself on the host; device code passes a copy held in
// constant memory, so the coefficients are scalar operands of the FMAs.
//
// With quadrant count n = 0 the reduction leaves x unchanged (a zero becomes
// +0, and the series maps either zero to sine +0 and cosine 1) and the
// fix-up below is the identity, so sincos_rad(x) has the bits of
// sincos_series(x) there; the kernels take that shortcut for whole waves.
__host__ __device__ inline void sincos_rad(double x, double *s, double *c, const SinCosCoef &k) {
    const double ax = fabs(x);
    if (!(ax < 131072.0)) {  // also catches NaN and infinities
        *s = ::sin(x);
        *c = ::cos(x);
        return;
    }
    constexpr double kPio2Hi = 1.5707963267948966192;     // pi/2 rounded to double
    constexpr double kPio2Lo = 6.123233995736766036e-17;  // pi/2 - kPio2Hi
    const double n = sincos_quadrant(x);
    double r = fma(-n, kPio2Hi, x);
    r = fma(-n, kPio2Lo, r);
    double sr, cr;
    sincos_series(r, &sr, &cr, k);
    const int qd = static_cast<int>(n) & 3;  // |n| < 2^17 here, so the conversion is exact
    const double so = (qd & 1) ? cr : sr;
    const double co = (qd & 1) ? sr : cr;
    *s = (qd & 2) ? -so : so;
    *c = ((qd + 1) & 2) ? -co : co;
}

}  // namespace pf
