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
//                   s = f / (2 + f), ln(1 + f) = 2 atanh(s) = 2 s + s R with
//                   R = z Q(z), z = s^2, Q(z) = 2 (atanh(s) - s) / s^3 a
//                   degree-6 Chebyshev fit, summed as f - (f^2/2 - s (f^2/2
//                   + R)) (the argument reduction and rearrangement of the
//                   classical fdlibm scheme); e ln 2 added with ln 2 split
//                   into a 33-bit head (exact product) and a tail.
//   exp(x):         Cody-Waite reduction x = k ln 2 + r, |r| <= ln(2) / 2,
//                   e^r = 1 + (r + r^2 P(r)) with P(r) = (e^r - 1 - r) / r^2
//                   a degree-10 Chebyshev fit, scaled by 2^k with ldexp.
//   log1p(x), x > -1: u = 1 + x rounded and its rounding error c; with
//                   u = m 2^e reduced as for ln, ln(1 + x) = e ln 2 +
//                   ln(1 + f') with f' = (m - 1) + c 2^-e, so the rounding
//                   of u never reaches the result.
//   expm1(x):       the same reduction, 2^k (e^r - 1) + (2^k - 1) with
//                   e^r - 1 = r + r^2 P(r).
//
// The fits come from gen_math_coeffs.py (qmc_math_coeffs.h), which checks
// each rounded polynomial against its error budget.  Errors are a few
// units in the last place, checked against the host library on wide
// samples by the tests.
//
// The float overloads (FP32 evaluation mode) build on the hardware base-2
// logarithm and exponential (v_log_f32, v_exp_f32: within 1 ulp over the
// normal range, arguments near 1 included, as measured on gfx950):
//   ln(x):          log2(x) times ln 2 as a head + tail product; subnormal
//                   x scaled by 2^32 first.
//   exp(x):         p = x log2(e) as a head + tail product, 2^p_head times
//                   1 + p_tail ln 2; results below the normal range formed
//                   as 2^(p + 64) 2^-64 so they round once.
//   log1p(x):       Goldberg's formulation ln(u) x / (u - 1) with u = 1 + x
//                   rounded (x itself when u = 1): the rounding of u cancels.
//   expm1(x):       Kahan's formulation (u - 1) x / ln(u) with u = e^x
//                   rounded (x itself when u = 1; u - 1 for |x| > 10).
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_math_coeffs.h"

namespace qmc_math {

// ln 2 = LN2_HI + LN2_LO, LN2_HI with 33 significant bits
constexpr double LN2_HI = 0x1.62e42fee00000p-1;
constexpr double LN2_LO = 0x1.a39ef35793c76p-33;
constexpr double LOG2E = 0x1.71547652b82fep+0;
constexpr double SQRT_HALF = 0x1.6a09e667f3bcdp-1;

// 1 / x for normal x: the hardware estimate and two Newton steps (one
// step leaves ~20 ulp: the estimate is good to about 2^-24; the tests bound
// the result at 2 ulp)
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// polynomial of degree N with coefficients c[0] (highest) .. c[N]
template <int N>
__device__ __forceinline__ double horner(const double (&c)[N + 1], double x)
{
    double p = c[0];
#pragma unroll
    for (int i = 1; i <= N; ++i) p = fma(p, x, c[i]);
    return p;
}

// ln(1 + f) for f in [sqrt(1/2) - 1, sqrt(2) - 1)
__device__ __forceinline__ double ln1pf_reduced(double f)
{
    const double s = f * rcp(2.0 + f);
    const double z = s * s;
    const double R = z * horner<LN_Q_DEG>(LN_Q, z);
    // ln(1 + f) = 2s + s R = f - s f + s R;  with hfsq = f^2 / 2 the
    // equivalent f - (hfsq - s (hfsq + R)) keeps the rounding of s small
    const double hfsq = 0.5 * f * f;
    return f - (hfsq - s * (hfsq + R));
}

// u = m 2^e with m in [sqrt(1/2), sqrt(2)), u > 0 finite
__device__ __forceinline__ void reduce_ln(double u, double &m, int &e)
{
    m = __builtin_amdgcn_frexp_mant(u);               // [1/2, 1)
    e = __builtin_amdgcn_frexp_exp(u);
    const bool lo = m < SQRT_HALF;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
}

// natural logarithm of a positive finite x
__device__ __forceinline__ double ln(double x)
{
    double m;
    int e;
    reduce_ln(x, m, e);
    const double k = (double)e;
    const double l = ln1pf_reduced(m - 1.0);          // m - 1 is exact
    return fma(k, LN2_HI, fma(k, LN2_LO, l));
}

// ln(1 + x) for x > -1: the rounding error c of u = 1 + x is added to the
// reduced argument, where it is scaled like u itself
__device__ __forceinline__ double ln1p(double x)
{
    const double u = 1.0 + x;
    const double c = x - (u - 1.0);                   // rounding error of u
    double m;
    int e;
    reduce_ln(u, m, e);
    const double f = (m - 1.0) + __builtin_amdgcn_ldexp(c, -e);
    const double k = (double)e;
    return fma(k, LN2_HI, fma(k, LN2_LO, ln1pf_reduced(f)));
}

// e^r - 1 for |r| <= ln(2) / 2
__device__ __forceinline__ double expm1_reduced(double r)
{
    return fma(r * r, horner<EXPM1_P_DEG>(EXPM1_P, r), r);
}

// e^x for finite x (results below the normal range may flush towards 0)
__device__ __forceinline__ double ex(double x)
{
    x = fmin(fmax(x, -1100.0), 710.0);
    const double k = __builtin_rint(x * LOG2E);
    double r = fma(-k, LN2_HI, x);
    r = fma(-k, LN2_LO, r);
    return __builtin_amdgcn_ldexp(1.0 + expm1_reduced(r), (int)k);
}

// e^x - 1 for finite x: with x = k ln 2 + r as in ex(),
// e^x - 1 = 2^k (e^r - 1) + (2^k - 1); 2^k - 1 is exact and the two terms
// never cancel by more than a factor of about 2.5.  k = 0 for
// |x| < ln(2) / 2, where the result is e^r - 1 itself.
__device__ __forceinline__ double exm1(double x)
{
    x = fmin(fmax(x, -80.0), 709.0);
    const double k = __builtin_rint(x * LOG2E);
    double r = fma(-k, LN2_HI, x);
    r = fma(-k, LN2_LO, r);
    const int ki = (int)k;
    return __builtin_amdgcn_ldexp(expm1_reduced(r), ki) + (__builtin_amdgcn_ldexp(1.0, ki) - 1.0);
}

constexpr float LN2F_HI = 0x1.62e430p-1f;       // ln 2 = LN2F_HI + LN2F_LO
constexpr float LN2F_LO = -0x1.05c610p-29f;
constexpr float LOG2EF_HI = 0x1.715476p+0f;     // log2(e) = LOG2EF_HI + LOG2EF_LO
constexpr float LOG2EF_LO = 0x1.4ae0c0p-26f;

// 1 / x: the hardware estimate and one Newton step
__device__ __forceinline__ float rcp(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// natural logarithm of a positive finite x
__device__ __forceinline__ float ln(float x)
{
    const bool sub = x < 0x1p-126f;
    float l = __builtin_amdgcn_logf(sub ? x * 0x1p32f : x);
    l = sub ? l - 32.0f : l;
    const float h = l * LN2F_HI;
    return h + fmaf(l, LN2F_LO, fmaf(l, LN2F_HI, -h));
}

// ln(1 + x) for x > -1
__device__ __forceinline__ float ln1p(float x)
{
    const float u = 1.0f + x;
    const float d = u - 1.0f;
    const float r = ln(u) * (x * rcp(d));
    return d == 0.0f ? x : r;
}

// e^x (0 below the subnormal range, inf above the float range)
__device__ __forceinline__ float ex(float x)
{
    x = fminf(fmaxf(x, -150.0f), 100.0f);
    const float p = x * LOG2EF_HI;
    const float e = fmaf(x, LOG2EF_LO, fmaf(x, LOG2EF_HI, -p));
    const bool sub = p < -126.0f;
    float r = __builtin_amdgcn_exp2f(sub ? p + 64.0f : p);
    r = fmaf(r, e * LN2F_HI, r);
    return sub ? r * 0x1p-64f : r;
}

// e^x - 1
__device__ __forceinline__ float exm1(float x)
{
    const float u = ex(x);
    const float d = u - 1.0f;
    if (!(fabsf(x) <= 10.0f)) return d;
    const float r = d * (x * rcp(ln(u)));
    return u == 1.0f ? x : r;
}

} // namespace qmc_math
