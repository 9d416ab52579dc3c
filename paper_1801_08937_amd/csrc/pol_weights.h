// Polarisation weights of one sample, Eq. datamodel: the pointing row of a
// sample at angle psi is (1, cos 2psi, sin 2psi).  Every kernel that forms
// the weights calls this one function, so weights computed on the fly and
// weights stored at pointing build are the same bits, and P and P^T stay
// exact transposes of each other.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

namespace detail {

// sin x and cos x for |x| <= 2^20, to within about one unit in the last
// place.  x = k pi/2 + r with k = rint(2x/pi), and r by two FMA steps against
// pi/2 split into a double and the rounding error of that double (the
// reduction of W. J. Cody and W. Waite, Software Manual for the Elementary
// Functions, 1980).  sin r and cos r on |r| <= pi/4 follow from their Taylor
// series through r^15 and r^16: the first omitted terms are below 5e-17.
// The quadrant k mod 4 then maps (sin r, cos r) to (sin x, cos x).  The
// constants are pi/2 and 2/pi rounded to double, the rounding error of pi/2,
// and the Taylor coefficients +-1/n! rounded to double.
__device__ __forceinline__ void sincos_reduced(double x, double &s, double &c) {
    constexpr double PIO2_HI = 1.5707963267948966;
    constexpr double PIO2_LO = 6.123233995736766e-17;
    constexpr double TWO_OVER_PI = 0.6366197723675814;
    const double kd = __builtin_rint(x * TWO_OVER_PI);
    double r = __builtin_fma(-kd, PIO2_HI, x);
    r = __builtin_fma(-kd, PIO2_LO, r);
    const double r2 = r * r;
    double ps = -7.647163731819816e-13;               // -1/15!
    ps = __builtin_fma(ps, r2, 1.6059043836821613e-10);  // 1/13!
    ps = __builtin_fma(ps, r2, -2.505210838544172e-08);  // -1/11!
    ps = __builtin_fma(ps, r2, 2.7557319223985893e-06);  // 1/9!
    ps = __builtin_fma(ps, r2, -0.0001984126984126984);  // -1/7!
    ps = __builtin_fma(ps, r2, 0.008333333333333333);    // 1/5!
    ps = __builtin_fma(ps, r2, -0.16666666666666666);    // -1/3!
    const double s0 = __builtin_fma(r * r2, ps, r);
    double pc = 4.779477332387385e-14;                   // 1/16!
    pc = __builtin_fma(pc, r2, -1.1470745597729725e-11); // -1/14!
    pc = __builtin_fma(pc, r2, 2.08767569878681e-09);    // 1/12!
    pc = __builtin_fma(pc, r2, -2.755731922398589e-07);  // -1/10!
    pc = __builtin_fma(pc, r2, 2.48015873015873e-05);    // 1/8!
    pc = __builtin_fma(pc, r2, -0.001388888888888889);   // -1/6!
    pc = __builtin_fma(pc, r2, 0.041666666666666664);    // 1/4!
    pc = __builtin_fma(pc, r2, -0.5);                    // -1/2!
    const double c0 = __builtin_fma(r2, pc, 1.0);
    const int q = (int)kd & 3;  // quadrant; two's complement keeps k mod 4 for k < 0
    const bool swap = (q & 1) != 0;
    s = swap ? c0 : s0;
    c = swap ? s0 : c0;
    if (q == 1 || q == 2) c = -c;
    if (q >= 2) s = -s;
}

}  // namespace detail

__device__ __forceinline__ void pol_weights(double psi, double &c, double &s) {
    const double x = 2.0 * psi;
    if (__builtin_fabs(x) <= 1048576.0)
        detail::sincos_reduced(x, s, c);
    else
        sincos(x, &s, &c);
}

}  // namespace mm
