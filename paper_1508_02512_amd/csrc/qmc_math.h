// Elementary functions for the integrand kernels.
//
// The integrand of Eq. 9 after the subtraction of Eq. 11 is dominated by
// logarithms (of the Feynman parameters and of U and F) and exponentials
// (monomials, the eps expansion).  The general-purpose device library
// versions handle infinities, NaNs and the whole exponent range and carry
// extra precision; the arguments here are finite and, for the logarithms,
// positive, so shorter sequences suffice:
//
//   ln(x), x > 0:   x = m 2^e with m in [sqrt(1/2), sqrt(2)), f = m - 1,
//                   s = f / (2 + f), ln(1 + f) = 2 atanh(s) written as
//                   f - s (f - R(s^2)) with the atanh series
//                   R(z) = sum_k 2 z^k / (2k + 1) (the argument reduction
//                   and rearrangement of the classical fdlibm scheme; here
//                   with the exact series coefficients, one more term than
//                   needed for |s| <= 3 - 2 sqrt(2): truncation < 1e-18);
//                   e ln 2 added with ln 2 split into a 33-bit head (exact
//                   product) and a tail.
//   exp(x):         Cody-Waite reduction x = k ln 2 + r, |r| <= ln(2) / 2,
//                   Taylor polynomial of degree 13 (truncation < 5e-18),
//                   scaled by 2^k with ldexp.
//   log1p(x), x > -1: u = 1 + x rounded, ln(u) corrected by the rounding
//                   error of u to first order, (x - (u - 1)) / u.
//   expm1(x):       the same reduction, 2^k (e^r - 1) + (2^k - 1) with the
//                   Taylor series of e^r - 1.
//
// Errors are a few units in the last place, checked against the host
// library on wide samples by the tests.  The float overloads (FP32
// evaluation mode) use the device library.
#pragma once

#include <hip/hip_runtime.h>

namespace qmc_math {

// ln 2 = LN2_HI + LN2_LO, LN2_HI with 33 significant bits
constexpr double LN2_HI = 0x1.62e42fee00000p-1;
constexpr double LN2_LO = 0x1.a39ef35793c76p-33;
constexpr double LOG2E = 0x1.71547652b82fep+0;
constexpr double SQRT_HALF = 0x1.6a09e667f3bcdp-1;

// 1 / x to about 1 ulp: the hardware estimate (relative error near 1e-8)
// and two Newton steps
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// ln(1 + f) for f in [sqrt(1/2) - 1, sqrt(2) - 1)
__device__ __forceinline__ double ln1pf_reduced(double f)
{
    const double s = f * rcp(2.0 + f);
    const double z = s * s;
    double R = 2.0 / 23.0;
    R = fma(R, z, 2.0 / 21.0);
    R = fma(R, z, 2.0 / 19.0);
    R = fma(R, z, 2.0 / 17.0);
    R = fma(R, z, 2.0 / 15.0);
    R = fma(R, z, 2.0 / 13.0);
    R = fma(R, z, 2.0 / 11.0);
    R = fma(R, z, 2.0 / 9.0);
    R = fma(R, z, 2.0 / 7.0);
    R = fma(R, z, 2.0 / 5.0);
    R = fma(R, z, 2.0 / 3.0);
    R *= z;
    // ln(1 + f) = 2s + s R = f - s f + s R;  with hfsq = f^2 / 2 the
    // equivalent f - (hfsq - s (hfsq + R)) keeps the rounding of s small
    const double hfsq = 0.5 * f * f;
    return f - (hfsq - s * (hfsq + R));
}

// natural logarithm of a positive finite x
__device__ __forceinline__ double ln(double x)
{
    double m = __builtin_amdgcn_frexp_mant(x);        // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool lo = m < SQRT_HALF;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double k = (double)e;
    const double l = ln1pf_reduced(m - 1.0);          // m - 1 is exact
    return fma(k, LN2_HI, fma(k, LN2_LO, l));
}

// ln(1 + x) for x > -1
__device__ __forceinline__ double ln1p(double x)
{
    const double u = 1.0 + x;
    const double c = x - (u - 1.0);                   // rounding error of u
    // for |x| below ulp(1) the correction is the whole result, so the
    // reciprocal must be accurate
    return ln(u) + c * rcp(u);
}

// e^x for finite x (results below the normal range may flush towards 0)
__device__ __forceinline__ double ex(double x)
{
    x = fmin(fmax(x, -1100.0), 710.0);
    const double k = __builtin_rint(x * LOG2E);
    double r = fma(-k, LN2_HI, x);
    r = fma(-k, LN2_LO, r);
    double p = 1.0 / 6227020800.0;               // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)k);
}

// e^x - 1 for finite x: with x = k ln 2 + r as in ex(),
// e^x - 1 = 2^k (e^r - 1) + (2^k - 1), e^r - 1 from its Taylor series of
// degree 14 (truncation < 3e-19 relative for |r| <= ln(2) / 2); 2^k - 1 is
// exact and the two terms never cancel by more than a factor of about 2.5.
// k = 0 for |x| < ln(2) / 2, where the result is the series itself.
__device__ __forceinline__ double exm1(double x)
{
    x = fmin(fmax(x, -80.0), 709.0);
    const double k = __builtin_rint(x * LOG2E);
    double r = fma(-k, LN2_HI, x);
    r = fma(-k, LN2_LO, r);
    double p = 1.0 / 87178291200.0;              // 1/14!, then down to 1/2
    p = fma(p, r, 1.0 / 6227020800.0);
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(r * r, p, r);                             // e^r - 1 = r + r^2 (1/2 + ...)
    const int ki = (int)k;
    return __builtin_amdgcn_ldexp(p, ki) + (__builtin_amdgcn_ldexp(1.0, ki) - 1.0);
}

__device__ __forceinline__ float ln(float x) { return logf(x); }
__device__ __forceinline__ float ln1p(float x) { return log1pf(x); }
__device__ __forceinline__ float ex(float x) { return expf(x); }
__device__ __forceinline__ float exm1(float x) { return expm1f(x); }

} // namespace qmc_math
