// Cancellation-free mixed differences for the pole subtraction of Eq. 11.
//
// With k poles the subtracted integrand needs, for every subset Y of the
// pole variables, the k-th order mixed difference
//     h^[Y] = sum_{Z subset Y} (-1)^{|Y \ Z|} h(t with the poles outside Z set to 0),
// the Moebius coefficient of the corner values of h.  Forming it from the
// corner values loses up to ~8 digits for k = 4 (the instability the paper
// points out before Eq. 13).  Here every quantity is carried as its vector
// of Moebius coefficients over the 2^k subsets instead:
//   - U and F: their coefficient for Y is the sum of the terms that contain
//     exactly the pole variables in Y, which is computed without
//     subtraction (the terms are grouped by that mask);
//   - products: h = f g has h^[Y] = sum_{A u B = Y} f^[A] g^[B];
//   - quotients q = a / b solve a^[Y] = q^[Y] b(Y) + sum_{A u B = Y, B != Y} b^[A] q^[B]
//     in increasing Y, with b(Y) the corner value;
//   - log(1 + x): splitting off the highest variable j,
//       log(1 + x)(W + j) - log(1 + x)(W) = log(1 + x_j / (1 + x_0))(W),
//     which recurses on one variable fewer and ends in scalar log1p.
// No step subtracts nearly equal quantities, so each coefficient keeps the
// relative accuracy of the working type T (double, or float in the FP32
// evaluation mode).  Index Y is a bit mask over the pole variables; all
// loops are over compile-time masks.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_math.h"

namespace mobius {

// reciprocal to ~1 ulp: the library's (hardware estimate, two Newton steps)
__device__ __forceinline__ double rcp(double x) { return qmc_math::rcp(x); }

__device__ __forceinline__ float rcp(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

// out = f * g (union product); only the coefficients with at most MAXPC
// variables are formed (the others are left untouched)
template <int KS, int MAXPC = KS, typename T>
__device__ __forceinline__ void mul(const T (&f)[1 << KS], const T (&g)[1 << KS],
                                    T (&out)[1 << KS])
{
    constexpr int N = 1 << KS;
#pragma unroll
    for (int Y = 0; Y < N; ++Y) {
        if (__builtin_popcount(Y) > MAXPC) continue;
        T s = 0;
#pragma unroll
        for (int A = 0; A < N; ++A) {
            if ((A & ~Y) != 0) continue;
            const int R = Y & ~A;
#pragma unroll
            for (int C = 0; C < N; ++C) {
                if ((C & ~A) != 0) continue;
                s = fma(f[A], g[R | C], s);
            }
        }
        out[Y] = s;
    }
}

// f <- f * g / (q + 1) in place, forming only the coefficients with at
// most MAXPC variables and zeroing the others.  A proper subset of Y has a
// smaller mask, so visiting Y in decreasing order reads every f^[A],
// A subset of Y, before it is overwritten.
template <int KS, int MAXPC, typename T>
__device__ __forceinline__ void mul_inplace(T (&f)[1 << KS], const T (&g)[1 << KS], T scale)
{
    constexpr int N = 1 << KS;
#pragma unroll
    for (int Y = N - 1; Y >= 0; --Y) {
        if (__builtin_popcount(Y) > MAXPC) {
            f[Y] = T(0);
            continue;
        }
        T s = 0;
#pragma unroll
        for (int A = 0; A < N; ++A) {
            if ((A & ~Y) != 0) continue;
            const int R = Y & ~A;
#pragma unroll
            for (int C = 0; C < N; ++C) {
                if ((C & ~A) != 0) continue;
                s = fma(f[A], g[R | C], s);
            }
        }
        f[Y] = s * scale;
    }
}

// corner value f(Y) = sum_{A subset Y} f^[A]
template <int KS, typename T>
__device__ __forceinline__ T corner(const T (&f)[1 << KS], int Y)
{
    T s = 0;
#pragma unroll
    for (int A = 0; A < (1 << KS); ++A)
        if ((A & ~Y) == 0) s += f[A];
    return s;
}

// q = a / b
template <int KS, typename T>
__device__ __forceinline__ void div(const T (&a)[1 << KS], const T (&b)[1 << KS],
                                    T (&q)[1 << KS])
{
    constexpr int N = 1 << KS;
#pragma unroll
    for (int Y = 0; Y < N; ++Y) {
        T s = a[Y];
#pragma unroll
        for (int A = 0; A < N; ++A) {
            if ((A & ~Y) != 0) continue;
            const int R = Y & ~A;
#pragma unroll
            for (int C = 0; C < N; ++C) {
                if ((C & ~A) != 0) continue;
                if ((R | C) == Y) continue;     // the unknown q^[Y] itself
                s = fma(-b[A], q[R | C], s);
            }
        }
        q[Y] = s * rcp(corner<KS, T>(b, Y));
    }
}

// Orders the two halves of a recursion in FP32: the values of v are made
// to depend on dep, so the second half starts after the first has
// finished.  The halves are independent, and interleaving them (the
// scheduler's choice) doubles the registers live at once.  Measured on the
// double box this helps the FP32 kernels (fewer spills at their higher
// occupancy); the FP64 ones lose more ILP than they gain, so there it is
// a no-op.
template <int N, typename T>
__device__ __forceinline__ void after(T (&v)[N], T dep)
{
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]) : "v"(dep));
    }
}

// Phase fence: every v[i] is made to depend on dep (the last value a phase
// produces), so no consumer of v starts before the whole phase is done.
template <int N, typename T>
__device__ __forceinline__ void fence(T (&v)[N], T dep)
{
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]) : "v"(dep));
}

// r = log(1 + x); with X0ZERO the caller guarantees x^[0] = 0, so the
// leaf on the empty set is 0 and is not evaluated
template <int KS, typename T, bool X0ZERO = false>
struct Log1p {
    static __device__ __forceinline__ void run(const T (&x)[1 << KS], T (&r)[1 << KS])
    {
        constexpr int H = 1 << (KS - 1);
        T x0[H], x1[H], d[H], y[H], r0[H], r1[H];
#pragma unroll
        for (int W = 0; W < H; ++W) {
            x0[W] = x[W];
            x1[W] = x[W + H];
            d[W] = x[W];
        }
        d[0] += T(1);
        Log1p<KS - 1, T, X0ZERO>::run(x0, r0);
        div<KS - 1, T>(x1, d, y);
        after<H, T>(y, r0[H - 1]);
        Log1p<KS - 1, T, false>::run(y, r1);
#pragma unroll
        for (int W = 0; W < H; ++W) {
            r[W] = r0[W];
            r[W + H] = r1[W];
        }
    }
};

template <typename T, bool X0ZERO>
struct Log1p<0, T, X0ZERO> {
    static __device__ __forceinline__ void run(const T (&x)[1], T (&r)[1])
    {
        r[0] = X0ZERO ? T(0) : qmc_math::ln1p(x[0]);
    }
};

// r = log(f) for f with a positive value at every corner
template <int KS, typename T>
__device__ __forceinline__ void log(const T (&f)[1 << KS], T (&r)[1 << KS])
{
    constexpr int N = 1 << KS;
    T x[N];
    const T inv0 = rcp(f[0]);
    x[0] = 0;
#pragma unroll
    for (int Y = 1; Y < N; ++Y) x[Y] = f[Y] * inv0;
    Log1p<KS, T, true>::run(x, r);
    r[0] = qmc_math::ln(f[0]);
}

// r = exp(x) - 1; with X0ZERO the caller guarantees x^[0] = 0
template <int KS, typename T, bool X0ZERO = false>
struct Expm1 {
    static __device__ __forceinline__ void run(const T (&x)[1 << KS], T (&r)[1 << KS])
    {
        constexpr int H = 1 << (KS - 1);
        T x0[H], x1[H], r0[H], r1[H], e0[H], p[H];
#pragma unroll
        for (int W = 0; W < H; ++W) {
            x0[W] = x[W];
            x1[W] = x[W + H];
        }
        Expm1<KS - 1, T, X0ZERO>::run(x0, r0);
        after<H, T>(x1, r0[H - 1]);
        Expm1<KS - 1, T, false>::run(x1, r1);
#pragma unroll
        for (int W = 0; W < H; ++W) e0[W] = r0[W];
        e0[0] += T(1);
        mul<KS - 1, KS - 1, T>(e0, r1, p);
#pragma unroll
        for (int W = 0; W < H; ++W) {
            r[W] = r0[W];
            r[W + H] = p[W];
        }
    }
};

template <typename T, bool X0ZERO>
struct Expm1<0, T, X0ZERO> {
    static __device__ __forceinline__ void run(const T (&x)[1], T (&r)[1])
    {
        r[0] = X0ZERO ? T(0) : qmc_math::exm1(x[0]);
    }
};

// r = exp(x)
template <int KS, typename T>
__device__ __forceinline__ void exp(const T (&x)[1 << KS], T (&r)[1 << KS])
{
    constexpr int N = 1 << KS;
    T y[N], e[N];
#pragma unroll
    for (int Y = 0; Y < N; ++Y) y[Y] = x[Y];
    y[0] = 0;
    Expm1<KS, T, true>::run(y, e);
    const T s = qmc_math::ex(x[0]);
    e[0] += T(1);
#pragma unroll
    for (int Y = 0; Y < N; ++Y) r[Y] = s * e[Y];
}

} // namespace mobius
