// Real (Euclidean) integrand kernel: shifted rank-1 lattice points generated
// in registers (Section III, Eqs. 17-18), Korobov periodiser (Eq. 21 at
// order r), sector integrand of Eq. 9 with the pole subtraction of Eq. 11
// and its eps expansion, compensated per-shift sums.
//
// One work-group of 256 lanes (four wave64) processes one work item: a tile
// of consecutive lattice indices of one (kinematic point, sector, shift).
// Sector data are wave-uniform (scalar loads, SGPRs) and the term loops are
// scalar loops; each lane owns one lattice point at a time and walks the
// tile with stride 256 by incremental modular addition.
//
// Monomials of U and F are products of powers: each lane writes t_j and
// t_j^2 into its own column of a work-group LDS table, and the host gives
// every term as words of four table slots (independent LDS reads and a
// product tree, against ~30 VALU operations for exp(sum_j e_j ln t_j),
// which remains the path for terms of very high degree).
//
// T is the evaluation type: double (QMC_FP64) or float (QMC_FP32_EVAL).
// Lattice points, the shift and the accumulation are FP64 in both.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_common.h"
#include "qmc_device.h"
#include "qmc_math.h"
#include "qmc_mobius.h"

namespace qmc_real {

using namespace qmc;

template <typename T>
__device__ __forceinline__ T tmono(uint32_t e, const T *t, const T *t2, const T *t3)
{
    T v = 1;
#pragma unroll
    for (int j = 0; j < QMC_DMAX; ++j) {
        const uint32_t ej = (e >> (4 * j)) & 15u;
        if (ej == 0u) continue;
        if (ej == 1u) {
            v *= t[j];
        } else if (ej == 2u) {
            v *= t2[j];
        } else if (ej == 3u) {
            v *= t3[j];
        } else {
            T p = t2[j] * t2[j];
            for (uint32_t k = 4u; k < ej; ++k) p *= t[j];
            v *= p;
        }
    }
    return v;
}

// prod_j t_j^e_j = exp(sum_j e_j ln t_j): branch-free for wave-uniform
// exponents (t_j > 0 wherever the real kernel evaluates a monomial)
template <typename T>
__device__ __forceinline__ T tmono_log(cptr<double> e, const T *lt, int d)
{
    T x = 0;
#pragma unroll
    for (int j = 0; j < QMC_DMAX; ++j)
        if (j < d) x = fma(T(e[j]), lt[j], x);
    return qmc_math::ex(x);
}

// sum_q c_q prod_j t_j^e_jq over one pole-mask group of terms: [q0, q1)
// with at most four power-table factors, [q1, q2) with five to eight,
// [q2, q3) in the exp form.  Factors are read from this lane's column of
// the power table at the byte offsets the planner stored per term (toff:
// the first four factors of every term, toff2: the next four), so the loops
// carry no branch and no decoding.  Terms of the first kind go in blocks of
// four: their 16 offsets arrive in one scalar load and their 16 LDS reads
// are in flight together.
template <typename T>
__device__ __forceinline__ T prod4_at(const char *colb, cptr<uint32_t> o)
{
    const T a = *(const T *)(colb + o[0]);
    const T b = *(const T *)(colb + o[1]);
    const T c = *(const T *)(colb + o[2]);
    const T e = *(const T *)(colb + o[3]);
    return (a * b) * (c * e);
}

template <typename T>
__device__ __forceinline__ T poly_group(int q0, int q1, int q2, int q3, cptr<uint32_t> toff,
                                        cptr<uint32_t> toff2, cptr<double> coef,
                                        const char *colb, cptr<double> texpd, const T *lt,
                                        int d)
{
    T s = 0;
    int q = q0;
    for (; q + 4 <= q1; q += 4) {
        cptr<uint32_t> o = toff + 4 * q;
        T v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = *(const T *)(colb + o[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            s = fma(T(coef[q + k]), (v[4 * k] * v[4 * k + 1]) * (v[4 * k + 2] * v[4 * k + 3]), s);
    }
    for (; q < q1; ++q) s = fma(T(coef[q]), prod4_at<T>(colb, toff + 4 * q), s);
    for (; q < q2; ++q)
        s = fma(T(coef[q]), prod4_at<T>(colb, toff + 4 * q) * prod4_at<T>(colb, toff2 + 4 * q), s);
    for (; q < q3; ++q) s = fma(T(coef[q]), tmono_log<T>(texpd + q * QMC_DMAX, lt, d), s);
    return s;
}

template <typename T>
__device__ __forceinline__ T tpowi(T x, int e)
{
    T r = 1;
    const int a = e < 0 ? -e : e;
    for (int k = 0; k < a; ++k) r *= x;
    return e < 0 ? mobius::rcp(r) : r;
}

template <typename T>
__device__ __forceinline__ void tkorobov(int r, T y, T u, T &t, T &w)
{
    if (r == 2) {
        t = y * y * y * fma(y, fma(T(6), y, T(-15)), T(10));
        w = T(30) * (y * u) * (y * u);
    } else if (r == 1) {
        t = y * y * fma(T(-2), y, T(3));
        w = T(6) * y * u;
    } else if (r == 3) {
        t = y * y * y * y * fma(y, fma(y, fma(T(-20), y, T(70)), T(-84)), T(35));
        const T yu = y * u;
        w = T(140) * yu * yu * yu;
    } else {
        t = y;
        w = 1;
    }
}

// Whether a sector with KS poles takes the Moebius-coefficient path
// (cancellation-free) rather than corner values: every sector with a pole.
template <typename T, int KS>
constexpr bool use_mobius()
{
    return KS >= 1;
}

template <int KS, int K, typename T>
struct Point {
    T SU[1 << KS];          // U, F coefficients per pole mask (Moebius coefficients)
    T SF[1 << KS];
    T E[KS > 0 ? KS : 1][K];   // (b_j ln t_j)^r / r! of the pole variables
    T invt[KS > 0 ? KS : 1];
    T lt[KS > 0 ? KS : 1];
    T LN;                   // sum_{j >= ks} b_j ln t_j
    int bad;                // U or F not positive at some corner
};

// ---- corner path (few poles) -------------------------------------------

template <int KS, int K, typename T>
__device__ __forceinline__ void leaf(cptr<qmc_sec_dev> S, Point<KS, K, T> &P, int X, T (&h)[K])
{
    constexpr int full = (1 << KS) - 1;
    const T u = P.SU[full ^ X];
    const T f = P.SF[full ^ X];
    P.bad |= !(u > T(0)) | !(f > T(0));
    const T lu = qmc_math::ln(u), lf = qmc_math::ln(f);
    T pre;
    if (S->u0i != QMC_NO_INT && S->f0i != QMC_NO_INT)
        pre = tpowi(u, S->u0i) * tpowi(f, S->f0i);
    else
        pre = qmc_math::ex(T(S->u0) * lu + T(S->f0) * lf);
    const T L = fma(T(S->u1), lu, fma(T(S->f1), lf, P.LN));
    h[0] = pre;
#pragma unroll
    for (int q = 1; q < K; ++q) h[q] = h[q - 1] * L * (T(1) / T(q));
}

// Fold one pole variable (Eq. 11 with alpha = -1):
//   G_R <- G_{R+j}/(b_j eps) + t_j^{-1} t_j^{b_j eps} (G_R - G_{R+j}),
// index q of the series staying order q - (folds done).
template <int K, typename T>
__device__ __forceinline__ void fold(T (&A)[K], const T (&B)[K], T invb, T invt, const T (&E)[K])
{
    T D[K];
#pragma unroll
    for (int q = 0; q < K; ++q) D[q] = A[q] - B[q];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        T s = 0;
#pragma unroll
        for (int r = 0; r < q; ++r) s = fma(E[r], D[q - 1 - r], s);
        A[q] = fma(B[q], invb, invt * s);
    }
}

template <int LEVEL, int XB, int KS, int K, typename T>
struct Tree {
    static __device__ __forceinline__ void run(cptr<qmc_sec_dev> S, Point<KS, K, T> &P,
                                               T (&out)[K])
    {
        T B[K];
        Tree<LEVEL - 1, XB, KS, K, T>::run(S, P, out);
        Tree<LEVEL - 1, XB | (1 << (LEVEL - 1)), KS, K, T>::run(S, P, B);
        fold<K, T>(out, B, T(S->inv_b[LEVEL - 1]), P.invt[LEVEL - 1], P.E[LEVEL - 1]);
    }
};

template <int XB, int KS, int K, typename T>
struct Tree<0, XB, KS, K, T> {
    static __device__ __forceinline__ void run(cptr<qmc_sec_dev> S, Point<KS, K, T> &P,
                                               T (&out)[K])
    {
        leaf<KS, K, T>(S, P, XB, out);
    }
};

// ---- Moebius path -----------------------------------------------------------

// g[q + r + |Y|] += C(Y) L(Y)^r / r! h_q^[Y] for each order q of h, with
// h_{q+1} = h_q B / (q + 1) formed only on the subsets that still
// contribute, C(Y) = prod_{j in Y} t_j^-1 prod_{j not in Y} 1/b_j and
// L(Y) = sum_{j in Y} b_j ln t_j (formed where used: fewer live registers).
// The factors of C(Y) are multiplied into h_q^[Y] one at a time: h^[Y]
// vanishes like prod_{j in Y} t_j, so every partial product stays of the
// size of the result, while C(Y) alone can exceed the float range (four
// poles at t_j ~ 1e-10).
//
// With PRE (FP64 builds with registers to spare) C(Y) and L(Y) are formed
// once per point, by subset products and sums, instead of at every order.
template <int KS, typename T>
struct SubsetConsts {
    T C[1 << KS], L[1 << KS];
};

template <int KS, int K, int Q, typename T, bool PRE>
struct Accum {
    static __device__ __forceinline__ void run(cptr<qmc_sec_dev> S, const Point<KS, K, T> &P,
                                               const T (&B)[1 << KS], T (&H)[1 << KS],
                                               T (&g)[K], const SubsetConsts<KS, T> &SC)
    {
        constexpr int N = 1 << KS;
#pragma unroll
        for (int Y = 0; Y < N; ++Y) {
            const int pc = __builtin_popcount(Y);
            if (Q + pc >= K) continue;
            T e = H[Y], L = 0;
            if constexpr (PRE) {
                e *= SC.C[Y];
                L = SC.L[Y];
            } else {
#pragma unroll
                for (int j = 0; j < KS; ++j) {
                    if (Y >> j & 1) {
                        e *= P.invt[j];
                        L = fma(T(S->b[j]), P.lt[j], L);
                    } else {
                        e *= T(S->inv_b[j]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int o = Q + r + pc;
                if (o < K) {
                    g[o] += e;
                    e *= L * (T(1) / T(r + 1));
                }
            }
        }
        if constexpr (Q + 1 < K) {
            constexpr int MAXPC = K - 2 - Q < KS ? K - 2 - Q : KS;
            // one level at a time (fences): overlapping this level's series
            // chains with the next level's product keeps both live
            mobius::fence<N, T>(H, g[K - 1]);
            mobius::mul_inplace<KS, MAXPC, T>(H, B, T(1) / T(Q + 1));
            mobius::fence<N, T>(H, H[0]);
            Accum<KS, K, Q + 1, T, PRE>::run(S, P, B, H, g, SC);
        }
    }
};

// The subtracted integrand from Moebius coefficients (see qmc_mobius.h):
// h = U^(u0+u1 eps) F^(f0+f1 eps) exp(eps LN) = exp(X) exp(eps B) with
// X = u0 log U + f0 log F and B = u1 log U + f1 log F + LN, accumulated into
//   g = sum_Y prod_{j not in Y} 1/(b_j eps) prod_{j in Y} t_j^-1 t_j^(b_j eps) h^[Y],
// index o of g holding order o - KS.
//
// With numerator factors (NUM, Eq. 13) h carries their product N as well:
// H = exp(X) is multiplied by N in the union algebra before the series.
template <int KS, int K, typename T, bool NUM, bool PRE>
__device__ __forceinline__ void mobius_series(cptr<qmc_sec_dev> S, Point<KS, K, T> &P,
                                              const T (&SN)[1 << KS], T (&g)[K])
{
    constexpr int N = 1 << KS;
#pragma unroll
    for (int Y = 0; Y < N; ++Y)
        P.bad |= !(mobius::corner<KS, T>(P.SU, Y) > T(0)) |
                 !(mobius::corner<KS, T>(P.SF, Y) > T(0));
    // log U is folded into B and X before log F is formed, so the two
    // logarithm vectors are never live together
    T B[N], H[N];
    {
        T X[N];
        {
            T l[N];
            mobius::log<KS, T>(P.SU, l);
#pragma unroll
            for (int Y = 0; Y < N; ++Y) {
                B[Y] = T(S->u1) * l[Y];
                X[Y] = T(S->u0) * l[Y];
            }
        }
        {
            T l[N];
            mobius::log<KS, T>(P.SF, l);
#pragma unroll
            for (int Y = 0; Y < N; ++Y) {
                B[Y] = fma(T(S->f1), l[Y], B[Y]);
                X[Y] = fma(T(S->f0), l[Y], X[Y]);
            }
        }
        B[0] += P.LN;
        // keep B and X formed here: otherwise the scheduler sinks their fmas
        // into the accumulation and both logarithm vectors stay live
#pragma unroll
        for (int Y = 0; Y < N; ++Y) asm volatile("" : "+v"(B[Y]), "+v"(X[Y]));
        mobius::exp<KS, T>(X, H);
        // the accumulation starts when the whole exponential is done:
        // overlapping the two keeps both phases' temporaries live
        mobius::fence<N, T>(H, H[N - 1]);
        if constexpr (NUM) {
            T R[N];
            mobius::mul<KS, KS, T>(H, SN, R);
#pragma unroll
            for (int Y = 0; Y < N; ++Y) H[Y] = R[Y];
        }
    }
    SubsetConsts<KS, T> SC;
    if constexpr (PRE) {
        // C(Y u {j}) = C(Y) b_j / t_j and L(Y u {j}) = L(Y) + b_j ln t_j
        SC.C[0] = T(1);
#pragma unroll
        for (int j = 0; j < KS; ++j) SC.C[0] *= T(S->inv_b[j]);
        SC.L[0] = T(0);
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const T cj = T(S->b[j]) * P.invt[j], lj = T(S->b[j]) * P.lt[j];
#pragma unroll
            for (int Y = 0; Y < (1 << j); ++Y) {
                SC.C[Y | (1 << j)] = SC.C[Y] * cj;
                SC.L[Y | (1 << j)] = SC.L[Y] + lj;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < K; ++o) g[o] = 0;
    Accum<KS, K, 0, T, PRE>::run(S, P, B, H, g, SC);
}

// Product of a sector's numerator factors (integration by parts, Eq. 13)
// as Moebius coefficients over the pole subsets: each factor's terms are
// grouped by pole mask like those of U, and the factors are multiplied in
// the union algebra (no subtraction, so no cancellation).
template <int KS, typename T>
__device__ __forceinline__ void numerator(cptr<qmc_sec_dev> S, cptr<uint32_t> toff,
                                          cptr<uint32_t> toff2, cptr<double> coef,
                                          const char *colb, cptr<double> texpd, const T *lt,
                                          int d, T (&SN)[1 << KS])
{
    constexpr int N = 1 << KS;
#pragma unroll
    for (int Y = 0; Y < N; ++Y) SN[Y] = T(Y == 0 ? 1 : 0);
    for (int i = 0; i < S->nf; ++i) {
        T SP[N], R[N];
#pragma unroll
        for (int m = 0; m < N; ++m)
            SP[m] = poly_group<T>(S->pm[i][m], S->pm1[i][m], S->pm2[i][m], S->pm[i][m + 1],
                                  toff, toff2, coef, colb, texpd, lt, d);
        mobius::mul<KS, KS, T>(SN, SP, R);
#pragma unroll
        for (int Y = 0; Y < N; ++Y) SN[Y] = R[Y];
    }
}

// ---- kernel -------------------------------------------------------------

// One work item (a tile of one (point, sector, shift) group).
// The three- and four-pole FP64 classes run at three and two waves per
// SIMD with more live values than registers.  Per-lane values that live
// across the whole point loop but are touched once per point are kept in
// LDS there instead, so the register allocator does not spill them to
// scratch: the compensated sums (both classes; three poles only while
// three work-groups still fit a CU's LDS) and the shift (four poles, where
// only two work-groups share a CU and LDS has room for it).
template <int KS, int K, typename T>
constexpr bool lds_sums()
{
    return sizeof(T) == 8 && (KS == 4 || (KS == 3 && K <= 4));
}

template <int KS, typename T>
constexpr bool lds_shift()
{
    return KS == 4 && sizeof(T) == 8;
}

template <int KS, int K, typename T>
constexpr int lds_state_slots()
{
    constexpr int n = (lds_sums<KS, K, T>() ? 2 * K : 0) + (lds_shift<KS, T>() ? QMC_DMAX : 0);
    return n > 0 ? n : 1;
}

template <int KS, int K, typename T, bool NUM, bool PRE>
__device__ __forceinline__ void qmc_eval_real_item(const qmc_launch_args &A, const int item_id,
                                                   T *col, double *st)
{
    const qmc_item it = load_item(A.items, item_id);
    cptr<qmc_sec_dev> S = ro(A.sec) + it.sector;
    cptr<qmc_lat_dev> L = ro(A.lat) + it.lat;
    const int d = S->dim;
    const uint32_t n = L->n;
    const double inv_n = L->inv_n;
    cptr<double> coef = ro(A.tcoef) + (size_t)it.point * A.n_terms;
    cptr<double> shift = ro(A.shifts) + it.shift * QMC_DMAX;
    cptr<double> texpd = ro(A.texpd);
    cptr<uint32_t> toff = ro(A.toff);
    cptr<uint32_t> toff2 = ro(A.toff) + (size_t)4 * A.n_terms;
    const int r = A.korobov_r;

    constexpr bool LDS = lds_sums<KS, K, T>();
    constexpr bool LDSH = lds_shift<KS, T>();
    // LDS slots of this lane (stride QMC_BLOCK): sums 0..K-1, compensations
    // K..2K-1, shift components 2K..2K+QMC_DMAX-1
    uint32_t l[QMC_DMAX], step[QMC_DMAX];
    double dl[QMC_DMAX];
#pragma unroll
    for (int j = 0; j < QMC_DMAX; ++j) {
        l[j] = 0u;
        step[j] = 0u;
        dl[j] = 0.0;
        if (j < d) {
            const uint64_t z = L->z[j];
            l[j] = (uint32_t)(((uint64_t)(it.start + it.stride * threadIdx.x) * z) % n);
            step[j] = (uint32_t)(((uint64_t)QMC_BLOCK * it.stride * z) % n);
            dl[j] = shift[S->perm[j]];
            if constexpr (LDSH) st[(2 * K + j) * QMC_BLOCK] = dl[j];
        }
    }

    double acc[1][K], cmp[1][K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        acc[0][q] = cmp[0][q] = 0.0;
        if constexpr (LDS) st[q * QMC_BLOCK] = st[(K + q) * QMC_BLOCK] = 0.0;
    }
    int viol = 0;

    const int np = (int)((it.count + QMC_BLOCK - 1) / QMC_BLOCK);
    for (int p = 0; p < np; ++p) {
        const uint32_t off = threadIdx.x + (uint32_t)p * QMC_BLOCK;
        if (off < it.count) {
            T t[QMC_DMAX], lt[QMC_DMAX], w = 1;
            bool skip = false;
#pragma unroll
            for (int j = 0; j < QMC_DMAX; ++j) {
                t[j] = 1;
                if (j < d) {
                    double dj = dl[j];
                    if constexpr (LDSH) dj = st[(2 * K + j) * QMC_BLOCK];
                    double y = fma((double)l[j], inv_n, dj);
                    if (y >= 1.0) y -= 1.0;
                    T wj;
                    tkorobov<T>(r, T(y), T(1.0 - y), t[j], wj);
                    w *= wj;
                    skip |= (t[j] == T(0));
                }
            }
            if (!(w == T(0) || skip)) {
                Point<KS, K, T> P;
                P.bad = 0;
                // non-pole monomial prod_{j >= ks} t_j^(a_j + b_j eps)
                T pn = 1, LN = 0;
#pragma unroll
                for (int j = 0; j < QMC_DMAX; ++j) {
                    lt[j] = 0;
                    if (j < d) {
                        constexpr int pole_lim = KS;
                        const bool pole = j < pole_lim;
                        const T bj = T(S->b[j]);
                        if (S->lnmask >> j & 1) lt[j] = qmc_math::ln(t[j]);
                        if (pole) {
                            const int jp = pole ? j : 0;
                            P.invt[jp] = mobius::rcp(t[j]);
                            P.lt[jp] = lt[j];
                            const T x = bj * lt[j];
                            P.E[jp][0] = 1;
#pragma unroll
                            for (int q = 1; q < K; ++q)
                                P.E[jp][q] = P.E[jp][q - 1] * x * (T(1) / T(q));
                        } else {
                            LN = fma(bj, lt[j], LN);
                            if (S->aint[j] == QMC_NO_INT) pn *= qmc_math::ex(T(S->a[j]) * lt[j]);
                            else
                                for (int k = 0; k < S->aint[j]; ++k) pn *= t[j];
                        }
                    }
                }
                P.LN = LN;
                // this lane's powers t_j, t_j^2 for the term programs; only
                // the lane itself reads its column, so no barrier is needed
#pragma unroll
                for (int j = 0; j < QMC_DMAX; ++j) {
                    if (j < d) {
                        col[(2 * j) * QMC_BLOCK] = t[j];
                        col[(2 * j + 1) * QMC_BLOCK] = t[j] * t[j];
                    }
                }
                // U and F: one pass over the terms grouped by pole mask
                const char *colb = (const char *)col;
#pragma unroll
                for (int m = 0; m < (1 << KS); ++m) {
                    P.SU[m] = poly_group<T>(S->um[m], S->um1[m], S->um2[m], S->um[m + 1], toff,
                                            toff2, coef, colb, texpd, lt, d);
                    P.SF[m] = poly_group<T>(S->fm[m], S->fm1[m], S->fm2[m], S->fm[m + 1], toff,
                                            toff2, coef, colb, texpd, lt, d);
                }
                T SN[1 << KS];
                if constexpr (NUM)
                    numerator<KS, T>(S, toff, toff2, coef, colb, texpd, lt, d, SN);
                T g[K];
                if constexpr (use_mobius<T, KS>()) {
                    mobius_series<KS, K, T, NUM, PRE>(S, P, SN, g);
                } else {
                    // subset sums: the value at the corner where the poles in X are 0
#pragma unroll
                    for (int i = 0; i < KS; ++i)
#pragma unroll
                        for (int Y = 0; Y < (1 << KS); ++Y)
                            if (Y >> i & 1) {
                                P.SU[Y] += P.SU[Y ^ (1 << i)];
                                P.SF[Y] += P.SF[Y ^ (1 << i)];
                            }
                    Tree<KS, 0, KS, K, T>::run(S, P, g);
                    if constexpr (NUM) {
#pragma unroll
                        for (int q = 0; q < K; ++q) g[q] *= SN[0];
                    }
                }
                // a term that is not finite (U or F not positive at a
                // corner, or an overflow) is counted, not summed
                bool finite = true;
#pragma unroll
                for (int q = 0; q < K; ++q) finite &= __builtin_isfinite(g[q]);
                if (P.bad || !finite) {
                    viol += 1;
                } else {
                    const double wp = (double)(w * pn);
                    if constexpr (LDS) {
#pragma unroll
                        for (int q = 0; q < K; ++q) {
                            double s = st[q * QMC_BLOCK], c = st[(K + q) * QMC_BLOCK];
                            neumaier(s, c, wp * (double)g[q]);
                            st[q * QMC_BLOCK] = s;
                            st[(K + q) * QMC_BLOCK] = c;
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < K; ++q)
                            neumaier(acc[0][q], cmp[0][q], wp * (double)g[q]);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < QMC_DMAX; ++j) {
            if (j < d) {
                const uint32_t v = l[j] + step[j];
                l[j] = v >= n ? v - n : v;
            }
        }
    }

    if constexpr (LDS) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            acc[0][q] = st[q * QMC_BLOCK];
            cmp[0][q] = st[(K + q) * QMC_BLOCK];
        }
    }
    double *dst = A.partial + (size_t)item_id * A.kstride * 4;
    block_reduce_store<K, 1>(acc, cmp, dst, A.kstride);
    store_violations(viol, A.viol + item_id);
}

// Work-groups take items item_begin + blockIdx.x, + gridDim.x, ...: one item
// per work-group when the grid covers the list, a persistent loop when the
// grid is smaller.  Each item writes only its own slot, so the result does
// not depend on the grid.
// Minimum waves per SIMD the register allocator must allow, i.e. how far
// it spills to buy occupancy.  Chosen per class from sweeps on the planar
// double box (n = 1000003, 4 shifts, ms per launch, FP64 / FP32):
//   poles 0: 4 waves (5.1 vs 6.1 ms at 3) / unconstrained
//   poles 1: 4 waves (41.3 vs 47.9 ms) / unconstrained
//   poles 2: 4 (57.7 vs 64.7 at 3 with the LDS power table; with exp-form
//            monomials 4 waves spilled 39 VGPRs and wrote ~390 GB of
//            scratch per launch) / 6 (45.7 vs 58.7)
//   poles 3: 3 (99.2; 2 gives 116.6, 4 gives 106.4) / 4 (73.3 vs 88.6)
//   poles 4: 2 (103.1; 1 gives 161.6, 3 gives 115.1) / 3 (82.2 vs 103.0)
template <int KS, typename T, int V>
constexpr int min_waves()
{
    constexpr int base = sizeof(T) == 8 ? (KS <= 2 ? 4 : (KS == 3 ? 3 : 2))
                                        : (KS <= 1 ? 1 : (KS == 2 ? 6 : (KS == 3 ? 4 : 3)));
    // occupancy variant 1: one wave fewer than the swept default, trading
    // latency hiding for fewer spills (the autotuner chooses per workload)
    return V == 0 ? base : (base > 1 ? base - 1 : 1);
}

template <int KS, int K, typename T, int V, bool NUM>
__global__ __launch_bounds__(QMC_BLOCK)
__attribute__((amdgpu_waves_per_eu(min_waves<KS, T, V>(), 8))) void qmc_eval_real(qmc_launch_args A)
{
    // per-lane power table: slot s of lane x at pw[s * QMC_BLOCK + x]; the
    // last slot is the constant 1 that pads the term programs
    __shared__ T pw[QMC_PROG_SLOTS * QMC_BLOCK];
    __shared__ double st[lds_state_slots<KS, K, T>() * QMC_BLOCK];
    pw[(QMC_PROG_SLOTS - 1) * QMC_BLOCK + threadIdx.x] = T(1);
    for (int item = A.item_begin + (int)blockIdx.x; item < A.item_end; item += (int)gridDim.x) {
        // FP64: the subset constants once per point (in FP32, C(Y) alone
        // can overflow, so there each factor is folded into h^[Y])
        constexpr bool PRE = sizeof(T) == 8 && KS >= 1;
        qmc_eval_real_item<KS, K, T, NUM, PRE>(A, item, pw + threadIdx.x, st + threadIdx.x);
        __syncthreads();
    }
}

} // namespace qmc_real

#define QMC_REAL_CASE(KS, KB, T, V, NUM)                                               \
    if (ks == KS && kb == KB) {                                                        \
        hipLaunchKernelGGL((qmc_real::qmc_eval_real<KS, KS + KB, T, V, NUM>), dim3(grid), \
                           dim3(QMC_BLOCK), 0, stream, args);                          \
        return hipGetLastError();                                                      \
    }

#define QMC_REAL_CASES_LO(T, V, NUM)                                                           \
    QMC_REAL_CASE(0, 1, T, V, NUM) QMC_REAL_CASE(0, 2, T, V, NUM) QMC_REAL_CASE(0, 3, T, V, NUM) \
    QMC_REAL_CASE(1, 1, T, V, NUM) QMC_REAL_CASE(1, 2, T, V, NUM) QMC_REAL_CASE(1, 3, T, V, NUM) \
    QMC_REAL_CASE(2, 1, T, V, NUM) QMC_REAL_CASE(2, 2, T, V, NUM) QMC_REAL_CASE(2, 3, T, V, NUM)

// pole-free sectors carrying 4-7 orders (integration by parts taken at the
// poles: the orders the poles would have held move above eps^0)
#define QMC_REAL_CASES_WIDE(T, V, NUM)                                                         \
    QMC_REAL_CASE(0, 4, T, V, NUM) QMC_REAL_CASE(0, 5, T, V, NUM) QMC_REAL_CASE(0, 6, T, V, NUM) \
    QMC_REAL_CASE(0, 7, T, V, NUM)

#define QMC_REAL_CASES_HI(T, V, NUM)                                                           \
    QMC_REAL_CASE(3, 1, T, V, NUM) QMC_REAL_CASE(3, 2, T, V, NUM) QMC_REAL_CASE(3, 3, T, V, NUM) \
    QMC_REAL_CASE(4, 1, T, V, NUM) QMC_REAL_CASE(4, 2, T, V, NUM) QMC_REAL_CASE(4, 3, T, V, NUM)
