// Integrand kernel with contour deformation (Section II, Eq. 14) for the
// physical region: every variable is deformed as
//     z_j = t_j - i lambda t_j (1 - t_j) dF/dt_j(t) = t_j phi_j,
// the Jacobian det(dz/dt) multiplies the integrand, and the sector integrand
// of Eq. 9 becomes
//     det J prod_j t_j^(a_j + b_j eps) phi_j^(a_j + b_j eps) U(z)^(u0+u1 eps) F(z)^(f0+f1 eps).
// F carries -i0: its logarithm takes the branch -i pi where F is real and
// negative.  Points where Im F(z) > 0 or Re U(z) <= 0 are counted as sign
// violations.  The pole subtraction of Eq. 11 uses the corner values of the
// deformed integrand (the deformation vanishes on t_j = 0 in z_j but not
// in the other variables, so every corner is a full evaluation).  The
// Jacobian determinant comes from an LDL^T factorisation of a complex
// symmetric matrix similar to dz/dt (see leaf()).
//
// T is the evaluation type of the polynomial work: double (QMC_FP64) or
// float (QMC_FP32_EVAL).  In float mode the power table, the gradient and
// Hessian terms of F, the deformed point z and the complex monomials of
// U(z) and F(z) are FP32; the Jacobian determinant, the logarithms and
// powers of U and F (F can come close to 0 on the contour), the eps series,
// the corner differences and the accumulation stay FP64.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_common.h"
#include "qmc_device.h"
#include "qmc_kernels.h"
#include "qmc_math.h"

namespace qmc_cplx {

using namespace qmc;

struct cd {
    double r, i;
};

__device__ __forceinline__ cd cmul(cd a, cd b)
{
    return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.r * s, a.i * s}; }

__device__ __forceinline__ cd crecip(cd a)
{
    const double inv = qmc_math::rcp(fma(a.r, a.r, a.i * a.i));
    return {a.r * inv, -a.i * inv};
}

__device__ __forceinline__ cd cpowi(cd x, int e)
{
    cd r = {1.0, 0.0};
    const int a = e < 0 ? -e : e;
    for (int k = 0; k < a; ++k) r = cmul(r, x);
    return e < 0 ? crecip(r) : r;
}

// principal logarithm; a real negative argument takes -i pi (the -i0 side)
__device__ __forceinline__ cd clog_m(cd x)
{
    const double m = 0.5 * qmc_math::ln(fma(x.r, x.r, x.i * x.i));
    double a = atan2(x.i, x.r);
    if (x.i == 0.0 && x.r < 0.0) a = -M_PI;
    return {m, a};
}

__device__ __forceinline__ cd cexp_(cd x)
{
    const double e = qmc_math::ex(x.r);
    double s, c;
    sincos(x.i, &s, &c);
    return {e * c, e * s};
}

// complex numbers in the evaluation type
template <typename T>
struct cx {
    T r, i;
};

template <typename T>
__device__ __forceinline__ cx<T> xmul(cx<T> a, cx<T> b)
{
    return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}

template <typename T>
__device__ __forceinline__ cd widen(cx<T> a)
{
    return {(double)a.r, (double)a.i};
}

// log(1 + q^2) / 2 and atan(q) in the evaluation type
__device__ __forceinline__ double half_log1p_sq(double q) { return 0.5 * qmc_math::ln1p(q * q); }
__device__ __forceinline__ float half_log1p_sq(float q) { return 0.5f * log1pf(q * q); }
__device__ __forceinline__ double atan_t(double q) { return atan(q); }
__device__ __forceinline__ float atan_t(float q) { return atanf(q); }

// prod_j z_j^e_j for 4-bit wave-uniform exponents, powers formed on the fly
// (no tables of z^2, z^3: the leaf's register budget goes to the Jacobian)
template <int DM, typename T>
__device__ __forceinline__ cx<T> cmonomial(uint32_t e, const cx<T> *z)
{
    cx<T> v = {T(1), T(0)};
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        const uint32_t ej = (e >> (4 * j)) & 15u;
        if (ej == 0u) continue;
        cx<T> p = z[j];
        if (ej >= 2u) {
            const cx<T> z2 = xmul(z[j], z[j]);
            p = ej == 2u ? z2 : xmul(z2, ej == 3u ? z[j] : z2);
            for (uint32_t k = 4u; k < ej; ++k) p = xmul(p, z[j]);
        }
        v = xmul(v, p);
    }
    return v;
}

template <int DM, typename T>
__device__ __forceinline__ T rmonomial(uint32_t e, const T *t)
{
    T v = 1;
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        const uint32_t ej = (e >> (4 * j)) & 15u;
        if (ej == 0u) continue;
        T p = t[j];
        if (ej >= 2u) {
            const T t2 = t[j] * t[j];
            p = ej == 2u ? t2 : t2 * (ej == 3u ? t[j] : t2);
            for (uint32_t k = 4u; k < ej; ++k) p *= t[j];
        }
        v *= p;
    }
    return v;
}

template <int DM, int KS, int K, typename T>
struct CplxPoint;

// derivative term q at the corner's real point: power-table product, or the
// branchy product of powers for terms with more than eight factors
template <int DM, int KS, int K, typename T>
__device__ __forceinline__ T dmono(const CplxPoint<DM, KS, K, T> &P, int q, const T *tp)
{
    return (P.dprog[2 * q] >> 31) ? rmonomial<DM, T>(P.dexp[q], tp)
                                  : tmono_lds<T>(P.dprog + 2 * q, P.col);
}

template <int DM, int KS, int K, typename T>
struct CplxPoint {
    double t[DM], omt[DM], lt[DM];
    double invt[KS > 0 ? KS : 1];
    double E[KS > 0 ? KS : 1][K];   // (b_j ln t_j)^r / r! of the pole variables
    double LN;                       // sum_{j >= ks} b_j ln t_j
    cptr<double> coef;               // U, F coefficients at this point
    cptr<double> dcoef;              // derivative coefficients at this point
    cptr<uint32_t> texp, dexp;
    cptr<uint32_t> dprog;            // derivative terms as power-table words
    T *col;                          // this lane's column of the power table
    double lam;                      // deformation parameter of this sector and point
    int bad;
};

// h at corner X (pole variables in X set to 0), deformed, as a series
template <int DM, int KS, int K, typename T>
__device__ __forceinline__ void leaf(cptr<qmc_sec_dev> S, CplxPoint<DM, KS, K, T> &P, int X,
                                     cd (&h)[K])
{
    T tp[DM], op[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        const bool zero = j < KS && ((X >> j) & 1);
        tp[j] = zero ? T(0) : T(P.t[j]);
        op[j] = zero ? T(1) : T(P.omt[j]);
    }
    const int d = S->dim;
    const T lam = T(P.lam);
    // powers of this corner's real point for the derivative terms (only
    // the lane itself reads its column)
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        if (j < d) {
            P.col[(2 * j) * QMC_BLOCK] = tp[j];
            P.col[(2 * j + 1) * QMC_BLOCK] = tp[j] * tp[j];
        }
    }
    // gradient of F at the real point
    T g[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        T s = 0;
        if (j < d)
            for (int q = S->d1[j]; q < S->d1[j + 1]; ++q)
                s = fma(T(P.dcoef[q]), dmono<DM, KS, K, T>(P, q, tp), s);
        g[j] = s;
    }
    // q_j = lambda (1 - t_j) g_j, phi_j = 1 - i q_j, z_j = t_j phi_j
    T qv[DM];
    cx<T> z[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        qv[j] = lam * op[j] * g[j];
        z[j] = {tp[j], -tp[j] * qv[j]};
    }
    // Jacobian dz/dt = I + i M with M = -lambda (T H + diag((1 - 2t) g)),
    // T = diag(t (1 - t)), H the Hessian of F.  With s_j = sqrt(lambda t_j
    // (1 - t_j)) the similarity S^-1 (I + i M) S gives
    //     det(dz/dt) = det(I + i A),  A = -S H S - lambda diag((1 - 2t) g),
    // A real symmetric: I + i A is complex symmetric with identity real
    // part, so an LDL^T factorisation without pivoting is stable.  Its lower
    // triangle is packed row by row; rows beyond the sector's dimension are
    // identity.  The factorisation is FP64 in both modes.
    T sj[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) sj[j] = j < d ? sqrt(lam * tp[j] * op[j]) : T(0);
    constexpr int NT = DM * (DM + 1) / 2;
    cd J[NT];
#pragma unroll
    for (int j = 0; j < DM; ++j) {
#pragma unroll
        for (int k = 0; k <= j; ++k) {
            T hs = 0;
            if (j < d) {
                const int idx = k * QMC_DMAX - k * (k - 1) / 2 + (j - k);
                for (int q = S->d2[idx]; q < S->d2[idx + 1]; ++q)
                    hs = fma(T(P.dcoef[q]), dmono<DM, KS, K, T>(P, q, tp), hs);
            }
            T a = -(sj[j] * hs) * sj[k];
            if (j == k && j < d) a -= lam * (op[j] - tp[j]) * g[j];
            J[j * (j + 1) / 2 + k] = {j == k ? 1.0 : 0.0, (double)a};
        }
    }
    cd det = {1.0, 0.0};
#pragma unroll
    for (int c = 0; c < DM; ++c) {
        const cd dc = J[c * (c + 1) / 2 + c];
        det = cmul(det, dc);
        const cd inv = crecip(dc);
#pragma unroll
        for (int r = c + 1; r < DM; ++r) {
            const cd f = cmul(J[r * (r + 1) / 2 + c], inv);
#pragma unroll
            for (int k = c + 1; k <= r; ++k)
                J[r * (r + 1) / 2 + k] = csub(J[r * (r + 1) / 2 + k], cmul(f, J[k * (k + 1) / 2 + c]));
        }
    }
    // U(z), F(z) in the evaluation type
    cx<T> Ut = {T(0), T(0)}, Ft = {T(0), T(0)};
    for (int q = S->um[0]; q < S->um[QMC_NMASK]; ++q) {
        const cx<T> v = cmonomial<DM, T>(P.texp[q], z);
        Ut.r = fma(T(P.coef[q]), v.r, Ut.r);
        Ut.i = fma(T(P.coef[q]), v.i, Ut.i);
    }
    for (int q = S->fm[0]; q < S->fm[QMC_NMASK]; ++q) {
        const cx<T> v = cmonomial<DM, T>(P.texp[q], z);
        Ft.r = fma(T(P.coef[q]), v.r, Ft.r);
        Ft.i = fma(T(P.coef[q]), v.i, Ft.i);
    }
    P.bad |= (Ft.i > T(0)) | !(Ut.r > T(0));
    // logarithms and powers of U and F in FP64
    const cd U = widen(Ut), F = widen(Ft);
    const cd lU = clog_m(U), lF = clog_m(F);
    cd pre;
    if (S->u0i != QMC_NO_INT && S->f0i != QMC_NO_INT)
        pre = cmul(cpowi(U, S->u0i), cpowi(F, S->f0i));
    else
        pre = cexp_(cadd(cscale(lU, S->u0), cscale(lF, S->f0)));
    pre = cmul(pre, det);
    cd L = cadd(cscale(lU, S->u1), cscale(lF, S->f1));
    L.r += P.LN;
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        if (j >= d || qv[j] == T(0)) continue;
        // Log phi_j = 1/2 log(1 + q^2) - i atan(q)
        const cd lphi = {(double)half_log1p_sq(qv[j]), -(double)atan_t(qv[j])};
        L = cadd(L, cscale(lphi, S->b[j]));
        const int ai = j < KS ? -1 : S->aint[j];
        if (ai == QMC_NO_INT)
            pre = cmul(pre, cexp_(cscale(lphi, S->a[j])));
        else if (ai != 0)
            pre = cmul(pre, cpowi(cd{1.0, -(double)qv[j]}, ai));
    }
    h[0] = pre;
#pragma unroll
    for (int q = 1; q < K; ++q) h[q] = cscale(cmul(h[q - 1], L), 1.0 / q);
}

template <int K>
__device__ __forceinline__ void cfold(cd (&A)[K], const cd (&B)[K], double invb, double invt,
                                      const double (&E)[K])
{
    cd D[K];
#pragma unroll
    for (int q = 0; q < K; ++q) D[q] = csub(A[q], B[q]);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int r = 0; r < q; ++r) {
            sr = fma(E[r], D[q - 1 - r].r, sr);
            si = fma(E[r], D[q - 1 - r].i, si);
        }
        A[q] = {fma(B[q].r, invb, invt * sr), fma(B[q].i, invb, invt * si)};
    }
}

// All corners of the pole variables in a runtime loop (the deformed leaf is
// large, so it is instantiated once); partial folds wait on a stack whose
// levels are unrolled: corner X completes level l when bit l of X is set.
template <int DM, int KS, int K, typename T>
__device__ __forceinline__ void corners_folded(cptr<qmc_sec_dev> S, CplxPoint<DM, KS, K, T> &P,
                                               cd (&out)[K])
{
    cd stack[KS > 0 ? KS : 1][K];
    for (int X = 0; X < (1 << KS); ++X) {
        cd cur[K];
        leaf<DM, KS, K, T>(S, P, X, cur);
        bool carry = true;
#pragma unroll
        for (int lev = 0; lev < KS; ++lev) {
            if (!carry) break;
            if ((X >> lev) & 1) {
                cd A[K];
#pragma unroll
                for (int q = 0; q < K; ++q) A[q] = stack[lev][q];
                cfold<K>(A, cur, S->inv_b[lev], P.invt[lev], P.E[lev]);
#pragma unroll
                for (int q = 0; q < K; ++q) cur[q] = A[q];
            } else {
#pragma unroll
                for (int q = 0; q < K; ++q) stack[lev][q] = cur[q];
                carry = false;
            }
        }
        if (carry) {
#pragma unroll
            for (int q = 0; q < K; ++q) out[q] = cur[q];
        }
    }
}

// One work item (a tile of one (point, sector, shift) group).
template <int DM, int KS, int K, typename T>
__device__ __forceinline__ void qmc_eval_cplx_item(const qmc_launch_args &A, const int item_id,
                                                   T *col)
{
    const qmc_item it = load_item(A.items, item_id);
    cptr<qmc_sec_dev> S = ro(A.sec) + it.sector;
    cptr<qmc_lat_dev> L = ro(A.lat) + it.lat;
    const int d = S->dim;
    const uint32_t n = L->n;
    const double inv_n = L->inv_n;
    cptr<double> shift = ro(A.shifts) + it.shift * QMC_DMAX;
    const int r = A.korobov_r;

    uint32_t l[DM], step[DM];
    double dl[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        l[j] = 0u;
        step[j] = 0u;
        dl[j] = 0.0;
        if (j < d) {
            const uint64_t zz = L->z[j];
            l[j] = (uint32_t)(((uint64_t)(it.start + it.stride * threadIdx.x) * zz) % n);
            step[j] = (uint32_t)(((uint64_t)QMC_BLOCK * it.stride * zz) % n);
            dl[j] = shift[S->perm[j]];
        }
    }
    double acc[2][K], cmp[2][K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[0][q] = acc[1][q] = cmp[0][q] = cmp[1][q] = 0.0;
    int viol = 0;

    const int np = (int)((it.count + QMC_BLOCK - 1) / QMC_BLOCK);
    for (int p = 0; p < np; ++p) {
        const uint32_t off = threadIdx.x + (uint32_t)p * QMC_BLOCK;
        if (off < it.count) {
            CplxPoint<DM, KS, K, T> P;
            P.coef = ro(A.tcoef) + (size_t)it.point * A.n_terms;
            P.dcoef = ro(A.dcoef) + (size_t)it.point * A.n_dterms;
            P.texp = ro(A.texp);
            P.dexp = ro(A.dexp);
            P.dprog = ro(A.dprog);
            P.col = col;
            P.lam = ro(A.lam)[(size_t)it.point * A.n_sec + it.sector];
            P.bad = 0;
            double w = 1.0;
            bool skip = false;
#pragma unroll
            for (int j = 0; j < DM; ++j) {
                P.t[j] = 1.0;
                P.omt[j] = 0.0;
                if (j < d) {
                    double y = fma((double)l[j], inv_n, dl[j]);
                    if (y >= 1.0) y -= 1.0;
                    double wj;
                    korobov(r, y, P.t[j], P.omt[j], wj);
                    w *= wj;
                    skip |= (P.t[j] == 0.0);
                }
            }
            if (!(w == 0.0 || skip)) {
                double pn = 1.0, LN = 0.0;
#pragma unroll
                for (int j = 0; j < DM; ++j) {
                    P.lt[j] = 0.0;
                    if (j < d) {
                        const bool pole = j < KS;
                        const double lt = qmc_math::ln(P.t[j]);
                        P.lt[j] = lt;
                        const double bj = S->b[j];
                        if (pole) {
                            P.invt[pole ? j : 0] = qmc_math::rcp(P.t[j]);
                            const double x = bj * lt;
                            P.E[pole ? j : 0][0] = 1.0;
#pragma unroll
                            for (int q = 1; q < K; ++q)
                                P.E[pole ? j : 0][q] = P.E[pole ? j : 0][q - 1] * x * (1.0 / q);
                        } else {
                            LN = fma(bj, lt, LN);
                            if (S->aint[j] == QMC_NO_INT) pn *= qmc_math::ex(S->a[j] * lt);
                            else
                                for (int k = 0; k < S->aint[j]; ++k) pn *= P.t[j];
                        }
                    }
                }
                P.LN = LN;
                cd g[K];
                corners_folded<DM, KS, K, T>(S, P, g);
                if (P.bad) {
                    viol += 1;
                } else {
                    const double wp = w * pn;
#pragma unroll
                    for (int q = 0; q < K; ++q) {
                        neumaier(acc[0][q], cmp[0][q], wp * g[q].r);
                        neumaier(acc[1][q], cmp[1][q], wp * g[q].i);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < DM; ++j) {
            if (j < d) {
                const uint32_t v = l[j] + step[j];
                l[j] = v >= n ? v - n : v;
            }
        }
    }
    double *dst = A.partial + (size_t)item_id * A.kstride * 4;
    block_reduce_store<K, 2>(acc, cmp, dst, A.kstride);
    store_violations(viol, A.viol + item_id);
}

// Work-groups take items item_begin + blockIdx.x, + gridDim.x, ...: one item
// per work-group when the grid covers the list, a persistent loop when the
// grid is smaller.  Each item writes only its own slot, so the result does
// not depend on the grid.
// The derivative terms (gradient and Hessian of F at each corner's real
// point) are products from a per-lane LDS power table, as in the real
// kernel; this cut the gg -> HH double boxes by 1.4x and the non-planar
// vertex by 1.5x against the branchy product of powers, which remains
// for the complex monomials of U and F (their table would not fit beside
// four work-groups per CU).
// The deformed integrand is bound by scalar work (wave-uniform term loops
// and exponent decoding) and its latency, so it is built for four waves per
// SIMD, which lets one wave's scalar and another's vector instructions issue
// together.  The register allocator spills 40-300 VGPRs per lane to
// scratch for that; measured on the gg -> HH double boxes and the
// non-planar vertex, one wave per SIMD (no spills) is 3.1x slower, two
// 1.9x, three 1.2x, six about the same, eight 1.15x.
// Occupancy variant 1 builds for two waves (far fewer spills); the
// autotuner chooses per workload.
template <int DM, int KS, int K, typename T, int V>
__global__ __launch_bounds__(QMC_BLOCK)
__attribute__((amdgpu_waves_per_eu(V == 0 ? 4 : 2, 8))) void qmc_eval_cplx(qmc_launch_args A)
{
    // per-lane power table of the corner points (slot layout as in the
    // real kernel, last slot the constant 1)
    __shared__ T pw[QMC_PROG_SLOTS * QMC_BLOCK];
    pw[(QMC_PROG_SLOTS - 1) * QMC_BLOCK + threadIdx.x] = T(1);
    for (int item = A.item_begin + (int)blockIdx.x; item < A.item_end; item += (int)gridDim.x) {
        qmc_eval_cplx_item<DM, KS, K, T>(A, item, pw + threadIdx.x);
        __syncthreads();
    }
}

} // namespace qmc_cplx

#define QMC_CPLX_CASE(DM, KS, KB, T, V)                                            \
    if (ks == KS && kb == KB) {                                                    \
        hipLaunchKernelGGL((qmc_cplx::qmc_eval_cplx<DM, KS, KS + KB, T, V>), dim3(grid), \
                           dim3(QMC_BLOCK), 0, stream, args);                      \
        return hipGetLastError();                                                  \
    }
