// pow64.hpp -- x^p for x >= 0 and p >= 1 in FP64 as 2^(p log2 x), for the
// L_p kinds whose p is neither an integer nor a half-integer.
//
// log2 x: x = m 2^e with m in [sqrt(1/2), sqrt(2)); with s = (m-1)/(m+1),
// ln m = 2 atanh(s) = 2 s sum_k s^(2k) / (2k+1), |s| <= 0.1716, so twelve
// terms (k = 0..11) leave a truncation below 2^-56. 2^f for f = y - rint(y)
// in [-1/2, 1/2]: exp(f ln 2) by its Taylor series to degree 14 (remainder
// below 2^-56), then scaled by 2^rint(y). Relative error, from the rounding
// of the series and of y = p log2 x: about (|y| + 8) * 2^-52; 0 gives 0,
// results beyond the FP64 range give 0 or inf.
#pragma once

#include <math.h>

#ifdef __HIPCC__
#define PCF_HD __host__ __device__
#else
#define PCF_HD
#endif

namespace pcf {

PCF_HD inline double log2_series(double x)
{
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    // sum_{k=0}^{11} z^k / (2k+1), Horner from the highest term
    double q = 1.0 / 23.0;
    q = fma(q, z, 1.0 / 21.0);
    q = fma(q, z, 1.0 / 19.0);
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    q = fma(q, z, 1.0);
    // log2 m = (2 / ln 2) s q
    const double two_over_ln2 = 2.88539008177792681472;
    return fma(two_over_ln2 * s, q, (double)e);
}

PCF_HD inline double exp2_series(double y)
{
    if (y < -1080.0)
        return 0.0;
    if (y > 1025.0)
        return INFINITY;
    const double n = rint(y);
    const double g = (y - n) * 0.69314718055994530942;  // f ln 2, |g| <= 0.3466
    // sum_{k=0}^{14} g^k / k!, Horner
    double r = 1.0 / 87178291200.0;
    r = fma(r, g, 1.0 / 6227020800.0);
    r = fma(r, g, 1.0 / 479001600.0);
    r = fma(r, g, 1.0 / 39916800.0);
    r = fma(r, g, 1.0 / 3628800.0);
    r = fma(r, g, 1.0 / 362880.0);
    r = fma(r, g, 1.0 / 40320.0);
    r = fma(r, g, 1.0 / 5040.0);
    r = fma(r, g, 1.0 / 720.0);
    r = fma(r, g, 1.0 / 120.0);
    r = fma(r, g, 1.0 / 24.0);
    r = fma(r, g, 1.0 / 6.0);
    r = fma(r, g, 0.5);
    r = fma(r, g, 1.0);
    r = fma(r, g, 1.0);
    return ldexp(r, (int)n);
}

PCF_HD inline double pow_series(double x, double p)
{
    return x == 0.0 ? 0.0 : exp2_series(p * log2_series(x));
}

}  // namespace pcf
