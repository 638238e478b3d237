// FP64 natural logarithm and exponential for the row update's power form of
// P = (W / S)^(1/gamma) (Sec. 2.1 Eq. (1) with the AdaIR exponent of Eq. (4)).
// P is rounded to FP32 once, so these need about 1e-13, not the last ulp of
// FP64, and are much shorter than general-purpose library functions.
//
// The header needs nothing but <cmath>: the device build includes it with
// HIP's math functions, and a host build (the CPU accuracy test) defines
// ACO_HD empty.  The reciprocal that seeds the logarithm's division is a
// parameter: the hardware FP64 reciprocal on the GPU, any approximation of
// 1/d to better than 2^-13 relative on the host.
#pragma once

#include <cmath>
#include <cstdint>

#ifndef ACO_HD
#define ACO_HD __host__ __device__
#endif

namespace aco {

// ln 2 in two parts (Cody and Waite): the high part has 24 trailing zero bits,
// so k * kLn2Hi is exact for every |k| < 2^24.
constexpr double kLn2Hi = 0x1.62e42ffp-1;
constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
constexpr double kLog2E = 0x1.71547652b82fep+0;

// Natural logarithm of a positive finite x.  With x = m 2^e, m in
// [sqrt(1/2), sqrt(2)), ln x = e ln 2 + 2 atanh(t) for t = (m - 1) / (m + 1),
// |t| < 0.172; the odd series of atanh is summed to t^19 (the first term left
// out is below 1e-17).  1 / (m + 1) comes from rcp and two Newton steps, each
// of which squares the relative error.  Absolute error below 1e-13 over the
// FP64 range.
template <typename Rcp>
ACO_HD inline double ln_positive(double x, Rcp rcp) {
    int e;
    double m = std::frexp(x, &e);  // [0.5, 1)
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double d = m + 1.0;
    double r = rcp(d);
    r = std::fma(r, std::fma(-d, r, 1.0), r);
    r = std::fma(r, std::fma(-d, r, 1.0), r);
    const double t = (m - 1.0) * r;
    const double s = t * t;
    double q = 1.0 / 19.0;
    q = std::fma(q, s, 1.0 / 17.0);
    q = std::fma(q, s, 1.0 / 15.0);
    q = std::fma(q, s, 1.0 / 13.0);
    q = std::fma(q, s, 1.0 / 11.0);
    q = std::fma(q, s, 1.0 / 9.0);
    q = std::fma(q, s, 1.0 / 7.0);
    q = std::fma(q, s, 1.0 / 5.0);
    q = std::fma(q, s, 1.0 / 3.0);
    q = std::fma(q, s, 1.0);
    const double de = static_cast<double>(e);
    return std::fma(de, kLn2Hi, std::fma(de, kLn2Lo, 2.0 * t * q));
}

// e^y for y <= 0 (or a rounding error above it), for a result that is then
// rounded to FP32: y = k ln 2 + r with k = rint(y / ln 2), |r| <= ln 2 / 2,
// e^r by its Taylor series to r^13 (the first term left out is below 4e-18),
// scaled by 2^k.  Below -200 it returns 0: e^-200 is far under half the
// smallest FP32 subnormal.  Relative error below 1e-15 elsewhere.
ACO_HD inline double exp_for_f32(double y) {
    if (y < -200.0) return 0.0;
    const double k = std::rint(y * kLog2E);
    double r = std::fma(-k, kLn2Hi, y);
    r = std::fma(-k, kLn2Lo, r);
    double p = 1.0 / 6227020800.0;
    p = std::fma(p, r, 1.0 / 479001600.0);
    p = std::fma(p, r, 1.0 / 39916800.0);
    p = std::fma(p, r, 1.0 / 3628800.0);
    p = std::fma(p, r, 1.0 / 362880.0);
    p = std::fma(p, r, 1.0 / 40320.0);
    p = std::fma(p, r, 1.0 / 5040.0);
    p = std::fma(p, r, 1.0 / 720.0);
    p = std::fma(p, r, 1.0 / 120.0);
    p = std::fma(p, r, 1.0 / 24.0);
    p = std::fma(p, r, 1.0 / 6.0);
    p = std::fma(p, r, 0.5);
    p = std::fma(p, r, 1.0);
    p = std::fma(p, r, 1.0);
    return std::ldexp(p, static_cast<int>(k));
}

}  // namespace aco
