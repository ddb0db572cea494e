// Integrand kernels for gfx950: shifted rank-1 lattice points generated in
// registers (Section III, Eqs. 17-18), Korobov periodiser (Eq. 21, order r),
// sector integrand of Eq. 9 with the pole subtraction of Eq. 11 and its eps
// expansion, and compensated per-shift sums.
//
// One work-group of 256 lanes (four wave64) processes one work item: a tile
// of consecutive lattice indices of one (kinematic point, sector, shift).
// All sector data are wave-uniform, so the compiler keeps them in SGPRs and
// the term loops are scalar loops; each lane owns one lattice point at a
// time and walks the tile with stride 256 by incremental modular addition.
#include <hip/hip_runtime.h>

#include "qmc_device.h"
#include "qmc_kernels.h"
#include "qmc_mobius.h"
#include "qmc_common.h"

namespace {

using namespace qmc;

// ------------------------------------------------------- real integrand

// Per-point state of the real (Euclidean) integrand.
template <int KS, int K>
struct RealPoint {
    double SU[1 << KS];      // U, F restricted to term masks, then at corners
    double SF[1 << KS];
    double E[KS > 0 ? KS : 1][K];   // (b_j ln t_j)^r / r!
    double invt[KS > 0 ? KS : 1];
    double LN;               // sum_{j >= ks} b_j ln t_j
    int bad;                 // U or F not positive at some corner
};

// h at corner X: U^(u0+u1 eps) F^(f0+f1 eps) exp(eps LN) as a series
template <int KS, int K>
__device__ __forceinline__ void leaf(const qmc_sec_dev *S, RealPoint<KS, K> &P,
                                     int X, double (&h)[K])
{
    constexpr int full = (1 << KS) - 1;
    const double u = P.SU[full ^ X];
    const double f = P.SF[full ^ X];
    P.bad |= !(u > 0.0) | !(f > 0.0);
    const double lu = log(u), lf = log(f);
    double pre;
    if (S->u0i != QMC_NO_INT && S->f0i != QMC_NO_INT)
        pre = ipow(u, S->u0i) * ipow(f, S->f0i);
    else
        pre = exp(S->u0 * lu + S->f0 * lf);
    const double L = fma(S->u1, lu, fma(S->f1, lf, P.LN));
    h[0] = pre;
#pragma unroll
    for (int q = 1; q < K; ++q) h[q] = h[q - 1] * L * (1.0 / q);
}

// Fold one pole variable (Eq. 11 with alpha = -1):
//   G_R <- G_{R+j}/(b_j eps) + t_j^{-1} t_j^{b_j eps} (G_R - G_{R+j}),
// with the series index shifted so that index q stays order q - (level).
template <int K>
__device__ __forceinline__ void fold(double (&A)[K], const double (&B)[K],
                                     double invb, double invt, const double (&E)[K])
{
    double D[K];
#pragma unroll
    for (int q = 0; q < K; ++q) D[q] = A[q] - B[q];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < q; ++r) s = fma(E[r], D[q - 1 - r], s);
        A[q] = fma(B[q], invb, invt * s);
    }
}

template <int LEVEL, int XB, int KS, int K>
struct Tree {
    static __device__ __forceinline__ void run(const qmc_sec_dev *S,
                                               RealPoint<KS, K> &P, double (&out)[K])
    {
        double B[K];
        Tree<LEVEL - 1, XB, KS, K>::run(S, P, out);
        Tree<LEVEL - 1, XB | (1 << (LEVEL - 1)), KS, K>::run(S, P, B);
        fold<K>(out, B, S->inv_b[LEVEL - 1], P.invt[LEVEL - 1], P.E[LEVEL - 1]);
    }
};

template <int XB, int KS, int K>
struct Tree<0, XB, KS, K> {
    static __device__ __forceinline__ void run(const qmc_sec_dev *S,
                                               RealPoint<KS, K> &P, double (&out)[K])
    {
        leaf<KS, K>(S, P, XB, out);
    }
};

// g[q + r + |Y|] += CY[Y] LY[Y]^r / r! h_q^[Y] for every order q of h, with
// h_{q+1} = h_q B / (q + 1) formed only where it still contributes.
template <int KS, int K, int Q>
struct Accum {
    static __device__ __forceinline__ void run(const qmc_sec_dev *S, const double (&B)[1 << KS],
                                               double (&T)[1 << KS], const double (&CY)[1 << KS],
                                               const double (&LY)[1 << KS], double (&g)[K])
    {
        constexpr int N = 1 << KS;
#pragma unroll
        for (int Y = 0; Y < N; ++Y) {
            const int pc = __builtin_popcount(Y);
            if (Q + pc >= K) continue;
            double e = CY[Y] * T[Y];
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int o = Q + r + pc;
                if (o < K) {
                    g[o] += e;
                    e *= LY[Y] * (1.0 / (r + 1));
                }
            }
        }
        if constexpr (Q + 1 < K) {
            constexpr int MAXPC = K - 2 - Q < KS ? K - 2 - Q : KS;
            double nt[N];
            mobius::mul<KS, MAXPC>(T, B, nt);
#pragma unroll
            for (int Y = 0; Y < N; ++Y)
                T[Y] = __builtin_popcount(Y) <= MAXPC ? nt[Y] * (1.0 / (Q + 1)) : 0.0;
            Accum<KS, K, Q + 1>::run(S, B, T, CY, LY, g);
        }
    }
};

// Sectors with two or more poles: the subtraction of Eq. 11 from Moebius
// coefficients (see qmc_mobius.h).  On entry P.SU, P.SF hold the mask sums
// of U and F, i.e. their Moebius coefficients.  h = U^(u0+u1 eps)
// F^(f0+f1 eps) exp(eps LN) = Pre exp(eps B) with B = u1 log U + f1 log F + LN;
// its coefficient h_q = Pre B^q / q! is accumulated into
//   g = sum_Y prod_{j not in Y} 1/(b_j eps) prod_{j in Y} t_j^-1 t_j^(b_j eps) h^[Y],
// index o of g holding order o - KS.
template <int KS, int K>
__device__ __forceinline__ void stable_series(const qmc_sec_dev *S, RealPoint<KS, K> &P,
                                              const double (&lt)[QMC_DMAX], double (&g)[K])
{
    constexpr int N = 1 << KS;
#pragma unroll
    for (int Y = 0; Y < N; ++Y)
        P.bad |= !(mobius::corner<KS>(P.SU, Y) > 0.0) | !(mobius::corner<KS>(P.SF, Y) > 0.0);
    double lU[N], lF[N], B[N], T[N];
    mobius::log<KS>(P.SU, lU);
    mobius::log<KS>(P.SF, lF);
#pragma unroll
    for (int Y = 0; Y < N; ++Y) B[Y] = fma(S->u1, lU[Y], S->f1 * lF[Y]);
    B[0] += P.LN;
    if (S->u0i != QMC_NO_INT && S->f0i != QMC_NO_INT) {
        double pu[N], pf[N];
        mobius::powi<KS>(P.SU, S->u0i, pu);
        mobius::powi<KS>(P.SF, S->f0i, pf);
        mobius::mul<KS>(pu, pf, T);
    } else {
        double x[N];
#pragma unroll
        for (int Y = 0; Y < N; ++Y) x[Y] = fma(S->u0, lU[Y], S->f0 * lF[Y]);
        mobius::exp<KS>(x, T);
    }
    // per subset: prod_{j in Y} 1/t_j * prod_{j not in Y} 1/b_j and sum_{j in Y} b_j ln t_j
    double CY[N], LY[N];
#pragma unroll
    for (int Y = 0; Y < N; ++Y) {
        double c = 1.0, L = 0.0;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            if (Y >> j & 1) {
                c *= P.invt[j];
                L = fma(S->b[j], lt[j], L);
            } else {
                c *= S->inv_b[j];
            }
        }
        CY[Y] = c;
        LY[Y] = L;
    }
#pragma unroll
    for (int o = 0; o < K; ++o) g[o] = 0.0;
    // h_q is needed only on subsets with at most K-1-q variables
    Accum<KS, K, 0>::run(S, B, T, CY, LY, g);
}

// ------------------------------------------------------------ kernels

template <int KS, int K>
__global__ __launch_bounds__(QMC_BLOCK) void qmc_eval_real(qmc_launch_args A)
{
    const int item_id = A.item_begin + (int)blockIdx.x;
    if (item_id >= A.item_end) return;
    const qmc_item it = A.items[item_id];
    const qmc_sec_dev *S = A.sec + it.sector;
    const qmc_lat_dev *L = A.lat + it.sector;
    const int d = S->dim;
    const uint32_t n = L->n;
    const double inv_n = L->inv_n;
    const double *coef = A.tcoef + (size_t)it.point * A.n_terms;
    const double *shift = A.shifts + it.shift * QMC_DMAX;
    const int r = A.korobov_r;

    uint32_t l[QMC_DMAX], step[QMC_DMAX];
    double dl[QMC_DMAX];
#pragma unroll
    for (int j = 0; j < QMC_DMAX; ++j) {
        l[j] = 0u;
        step[j] = 0u;
        dl[j] = 0.0;
        if (j < d) {
            const uint64_t z = L->z[j];
            l[j] = (uint32_t)(((uint64_t)(it.start + threadIdx.x) * z) % n);
            step[j] = (uint32_t)(((uint64_t)QMC_BLOCK * z) % n);
            dl[j] = shift[S->perm[j]];
        }
    }

    double acc[1][K], cmp[1][K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[0][q] = cmp[0][q] = 0.0;
    int viol = 0;

    for (int p = 0; p < A.ppl; ++p) {
        const uint32_t off = threadIdx.x + (uint32_t)p * QMC_BLOCK;
        if (off < it.count) {
            double t[QMC_DMAX], t2[QMC_DMAX], t3[QMC_DMAX], w = 1.0;
            bool skip = false;
#pragma unroll
            for (int j = 0; j < QMC_DMAX; ++j) {
                t[j] = 1.0;
                if (j < d) {
                    double y = fma((double)l[j], inv_n, dl[j]);
                    if (y >= 1.0) y -= 1.0;
                    double omt, wj;
                    korobov(r, y, t[j], omt, wj);
                    w *= wj;
                    skip |= (t[j] == 0.0);
                }
                t2[j] = t[j] * t[j];
                t3[j] = t2[j] * t[j];
            }
            if (!(w == 0.0 || skip)) {
                RealPoint<KS, K> P;
                P.bad = 0;
                double ltp[QMC_DMAX];
                // non-pole monomial prod_{j >= ks} t_j^(a_j + b_j eps)
                double pn = 1.0, LN = 0.0;
#pragma unroll
                for (int j = 0; j < QMC_DMAX; ++j) {
                    if (j < d) {
                        const bool pole = j < KS;
                        const double bj = S->b[j];
                        if (pole || bj != 0.0 || S->aint[j] == QMC_NO_INT) {
                            const double lt = log(t[j]);
                            ltp[j] = lt;
                            if (pole) {
                                P.invt[pole ? j : 0] = 1.0 / t[j];
                                const double x = bj * lt;
                                P.E[pole ? j : 0][0] = 1.0;
#pragma unroll
                                for (int q = 1; q < K; ++q)
                                    P.E[pole ? j : 0][q] = P.E[pole ? j : 0][q - 1] * x * (1.0 / q);
                            } else {
                                LN = fma(bj, lt, LN);
                                if (S->aint[j] == QMC_NO_INT) pn *= exp(S->a[j] * lt);
                            }
                        }
                        if (!pole && S->aint[j] != QMC_NO_INT)
                            for (int k = 0; k < S->aint[j]; ++k) pn *= t[j];
                    }
                }
                P.LN = LN;
                // U and F: one pass over the terms grouped by pole mask
#pragma unroll
                for (int m = 0; m < (1 << KS); ++m) {
                    double su = 0.0, sf = 0.0;
                    for (int q = S->um[m]; q < S->um[m + 1]; ++q)
                        su = fma(coef[q], monomial(A.texp[q], t, t2, t3), su);
                    for (int q = S->fm[m]; q < S->fm[m + 1]; ++q)
                        sf = fma(coef[q], monomial(A.texp[q], t, t2, t3), sf);
                    P.SU[m] = su;
                    P.SF[m] = sf;
                }
                double g[K];
                if constexpr (KS >= 2) {
                    stable_series<KS, K>(S, P, ltp, g);
                } else {
                    // subset sums: value at the corner where the poles in X are 0
#pragma unroll
                    for (int i = 0; i < KS; ++i)
#pragma unroll
                        for (int Y = 0; Y < (1 << KS); ++Y)
                            if (Y >> i & 1) {
                                P.SU[Y] += P.SU[Y ^ (1 << i)];
                                P.SF[Y] += P.SF[Y ^ (1 << i)];
                            }
                    Tree<KS, 0, KS, K>::run(S, P, g);
                }
                const double wp = w * pn;
                if (P.bad) {
                    viol += 1;
                } else {
#pragma unroll
                    for (int q = 0; q < K; ++q) neumaier(acc[0][q], cmp[0][q], wp * g[q]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < QMC_DMAX; ++j) {
            if (j < d) {
                uint32_t v = l[j] + step[j];
                l[j] = v >= n ? v - n : v;
            }
        }
    }

    double *dst = A.partial + (size_t)item_id * A.kstride * 4;
    block_reduce_store<K, 1>(acc, cmp, dst, A.kstride);
    store_violations(viol, A.viol + item_id);
}

} // namespace

// ------------------------------------------------------------- dispatch

#define QMC_REAL_CASE(KS, KB)                                                   \
    if (ks == KS && kb == KB) {                                                 \
        hipLaunchKernelGGL((qmc_eval_real<KS, KS + KB>), dim3(grid), dim3(QMC_BLOCK), 0, \
                           stream, args);                                       \
        return hipGetLastError();                                               \
    }

hipError_t qmc_launch_real(int ks, int kb, const qmc_launch_args &args, int grid,
                           hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    QMC_REAL_CASE(0, 1) QMC_REAL_CASE(0, 2) QMC_REAL_CASE(0, 3)
    QMC_REAL_CASE(1, 1) QMC_REAL_CASE(1, 2) QMC_REAL_CASE(1, 3)
    QMC_REAL_CASE(2, 1) QMC_REAL_CASE(2, 2) QMC_REAL_CASE(2, 3)
    QMC_REAL_CASE(3, 1) QMC_REAL_CASE(3, 2) QMC_REAL_CASE(3, 3)
    QMC_REAL_CASE(4, 1) QMC_REAL_CASE(4, 2) QMC_REAL_CASE(4, 3)
    return hipErrorInvalidValue;
}

// Fixed-order compensated sum of the tiles of every output group.
__global__ void qmc_reduce_groups(const double *partial, const int32_t *viol,
                                  const int32_t *group_begin, const int32_t *group_end,
                                  int n_groups, int kstride, double *out, int32_t *gviol)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = (int)(tid / kstride), q = (int)(tid % kstride);
    if (g >= n_groups) return;
    const int i0 = group_begin[g], i1 = group_end[g];
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    int v = 0;
    for (int i = i0; i < i1; ++i) {
        const double *p = partial + ((size_t)i * kstride + q) * 4;
        double e;
        two_sum(sr, p[0], sr, e);
        cr += p[1] + e;
        two_sum(si, p[2], si, e);
        ci += p[3] + e;
        if (q == 0) v += viol[i];
    }
    out[((size_t)g * kstride + q) * 2] = sr + cr;
    out[((size_t)g * kstride + q) * 2 + 1] = si + ci;
    if (q == 0) gviol[g] = v;
}

hipError_t qmc_launch_reduce(const double *partial, const int32_t *viol,
                             const int32_t *group_begin, const int32_t *group_end,
                             int n_groups, int kstride, double *out, int32_t *gviol,
                             hipStream_t stream)
{
    const long total = (long)n_groups * kstride;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (int)((total + threads - 1) / threads);
    hipLaunchKernelGGL(qmc_reduce_groups, dim3(blocks), dim3(threads), 0, stream,
                       partial, viol, group_begin, group_end, n_groups, kstride, out,
                       gviol);
    return hipGetLastError();
}
