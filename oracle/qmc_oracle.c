/*
 * Oracle: shifted rank-1 lattice sum of one sector integrand, in FP64.
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library; the GPU path never does.
 *
 * For one sector of the form of Eq. 9 (Section II),
 *
 *   I = int_[0,1]^d  prod_j t_j^(a_j + b_j eps)  P_1(t) .. P_r(t)
 *                     U(t)^(u0 + u1 eps)  F(t)^(f0 + f1 eps) dt
 *
 * (the numerator factors P_i, polynomials of any sign, come from the
 * integration by parts of Eq. 13; r = 0 for the sectors of Eq. 9)
 * and every shift k it returns the shifted lattice sums (Section III,
 * Eqs. 17-18, before the 1/n)
 *
 *   S_k(eps) = sum_{i=0}^{n-1} w(y) g(t(y)),   y = { i z / n + Delta_k },
 *
 * truncated to the requested Laurent orders, with
 *   - the periodising transform of Eq. 21, generalised to the Korobov
 *     order r: t = psi_r(y) = int_0^y u^r (1-u)^r du / B(r+1, r+1), weight
 *     w = prod_j y_j^r (1-y_j)^r / B(r+1, r+1)  (r = 1 is the paper's
 *     3y^2 - 2y^3; 1 - t is computed as psi_r(1 - y));
 *   - the pole subtraction of Eq. 11 (alpha = -1 only) applied to every
 *     variable with a_j = -1 in turn, which expands to
 *       g = sum_{R subset J} prod_{j in R} 1/(b_j eps)
 *             prod_{j in J\R} t_j^(-1 + b_j eps)
 *             sum_{S subset J\R} (-1)^|S| h(t with t_{R u S} = 0);
 *   - the contour deformation of Eq. 14 when lambda > 0, applied to every
 *     variable with the gradient of the sector's F:
 *       z_j = t_j - i lambda t_j (1 - t_j) dF/dt_j(t),
 *     so h = det(dz/dt) prod_{j not in J} z_j^(a_j + b_j eps)
 *            prod_{j in J} (z_j/t_j)^(-1 + b_j eps) U(z)^(..) F(z)^(..).
 *     F carries -i0: where Im F = 0 and Re F < 0, log F = ln|F| - i pi.
 *
 * Sums use Neumaier compensation in chunks of 2^16 consecutive indices,
 * combined in chunk order, so the result does not depend on the thread
 * count.  A point where the weight is 0 or some t_j is exactly 0
 * contributes 0.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Working precision of the integrand.  The default build is FP64.  The
 * subtraction of Eq. 11 with k poles forms k-th mixed differences of the
 * integrand, which amplifies rounding by up to ~1e8 for k = 4; the build
 * with -DORACLE_QUAD evaluates the same formula in IEEE binary128
 * (libquadmath) so that the oracle's own rounding stays far below FP64
 * roundoff of the result.  Lattice points, weights and sums stay FP64.
 */
#ifdef ORACLE_QUAD
#include <quadmath.h>
typedef __float128 real;
typedef __complex128 cplx;
#define RLOG logq
#define CLOG clogq
#define CEXP cexpq
#define CABS cabsq
#define CREAL crealq
#define CIMAG cimagq
#define RPI M_PIq
#define SYM(name) name##_q
#else
typedef double real;
typedef double complex cplx;
#define RLOG log
#define CLOG clog
#define CEXP cexp
#define CABS cabs
#define CREAL creal
#define CIMAG cimag
#define RPI M_PI
#define SYM(name) name
#endif

#define ORD_LO (-10)            /* lowest representable order */
#define ORD_N 24                /* orders ORD_LO .. ORD_LO+ORD_N-1 */
#define MAXD 16
#define CHUNK (1u << 16)

typedef struct {
    int dim;
    const double *a, *b;        /* [dim] */
    int nU;
    const int32_t *eU;          /* [nU][dim] */
    const double *cU;           /* [nU] */
    int nF;
    const int32_t *eF;
    const double *cF;
    double u0, u1, f0, f1;
    int nP;                     /* numerator factors */
    const int32_t *nPt;         /* [nP] terms of each factor */
    const int32_t *eP;          /* [sum nPt][dim], factor by factor */
    const double *cP;           /* [sum nPt] */
} oracle_sector;

/* A truncated Laurent series: c[q] is the coefficient of eps^(ORD_LO+q);
 * orders above `top` are dropped by every operation. */
typedef struct { cplx c[ORD_N]; } series;

/* Orders kept by the series operations of one call: top is the highest
 * order kept, bot the lowest that can be non-zero.  Passed explicitly, so
 * concurrent calls from different host threads do not interfere. */
typedef struct { int top, bot; } lims;

static void s_zero(series *s) { memset(s, 0, sizeof *s); }

static void s_const(series *s, cplx v) { s_zero(s); s->c[-ORD_LO] = v; }

/* product, truncated above L->top; every factor is zero below L->bot */
static void s_mul(const lims *L, series *out, const series *x, const series *y)
{
    series r;
    s_zero(&r);
    const int lo = L->bot - ORD_LO, hi = L->top - ORD_LO;
    for (int p = lo; p <= hi; ++p) {
        if (x->c[p] == 0) continue;
        for (int q = lo; q <= hi; ++q) {
            int o = p + q + ORD_LO;     /* index of order (p+LO)+(q+LO) */
            if (o < 0 || o > hi) continue;
            r.c[o] += x->c[p] * y->c[q];
        }
    }
    *out = r;
}

static void s_axpy(const lims *L, series *acc, cplx alpha, const series *x)
{
    for (int p = L->bot - ORD_LO; p <= L->top - ORD_LO; ++p) acc->c[p] += alpha * x->c[p];
}

/* exp(v eps) as a series */
static void s_exp_eps(const lims *L, series *s, cplx v)
{
    s_zero(s);
    cplx term = 1;
    for (int k = 0; k <= L->top && -ORD_LO + k < ORD_N; ++k) {
        s->c[-ORD_LO + k] = term;
        term = term * v / (real)(k + 1);
    }
}

/* x^(p + q eps) = exp(p L) exp(q eps L) with L the logarithm below */
static cplx logF(cplx x)
{
    if (CIMAG(x) == 0 && CREAL(x) < 0)
        return RLOG(-CREAL(x)) - I * RPI;      /* the -i0 side */
    return CLOG(x);
}

static void s_pow(const lims *lim, series *s, cplx x, double p, double q)
{
    cplx L = logF(x);
    s_exp_eps(lim, s, (real)q * L);
    cplx base = CEXP((real)p * L);
    for (int k = 0; k < ORD_N; ++k) s->c[k] *= base;
}

/* 1/(b eps) * x */
static void s_div_eps(series *out, const series *x, double b)
{
    series r;
    s_zero(&r);
    for (int p = 1; p < ORD_N; ++p) r.c[p - 1] = x->c[p] / (real)b;
    *out = r;
}

static real ipow(real x, int e)
{
    real r = 1;
    for (int k = 0; k < e; ++k) r *= x;
    return r;
}

static cplx cipow(cplx x, int e)
{
    cplx r = 1;
    for (int k = 0; k < e; ++k) r *= x;
    return r;
}

/* Korobov periodiser of order r (Eq. 21 for r = 1). */
static double beta_inv(int r)   /* 1/B(r+1,r+1) = (2r+1)!/(r!)^2 */
{
    double f = 1.0;
    for (int k = r + 1; k <= 2 * r + 1; ++k) f *= k;
    for (int k = 1; k <= r; ++k) f /= k;
    return f;
}

static double psi_r(double y, int r)
{
    double s = 0.0, binom = 1.0;
    for (int k = 0; k <= r; ++k) {
        s += ((k & 1) ? -binom : binom) * pow(y, r + k + 1) / (r + k + 1);
        binom = binom * (r - k) / (k + 1);
    }
    return s * beta_inv(r);
}

static double omega_r(double y, int r)
{
    return pow(y * (1.0 - y), r) * beta_inv(r);
}

static cplx poly_cplx(int n, const int32_t *e, const double *c, int d,
                      const cplx *z)
{
    cplx s = 0;
    for (int a = 0; a < n; ++a) {
        cplx v = (real)c[a];
        for (int j = 0; j < d; ++j) v *= cipow(z[j], e[a * d + j]);
        s += v;
    }
    return s;
}

/* first derivative d/dt_j of the polynomial at t */
static real poly_d1(int n, const int32_t *e, const double *c, int d,
                    const real *t, int j)
{
    real s = 0;
    for (int a = 0; a < n; ++a) {
        int ej = e[a * d + j];
        if (ej == 0) continue;
        real v = (real)c[a] * ej;
        for (int l = 0; l < d; ++l)
            v *= ipow(t[l], e[a * d + l] - (l == j));
        s += v;
    }
    return s;
}

/* second derivative d^2/dt_j dt_k */
static real poly_d2(int n, const int32_t *e, const double *c, int d,
                    const real *t, int j, int k)
{
    real s = 0;
    for (int a = 0; a < n; ++a) {
        int ej = e[a * d + j], ek = e[a * d + k];
        real v = (real)c[a];
        if (j == k) {
            if (ej < 2) continue;
            v *= ej * (ej - 1);
        } else {
            if (ej == 0 || ek == 0) continue;
            v *= ej * ek;
        }
        for (int l = 0; l < d; ++l) {
            int drop = (l == j) + (l == k);
            v *= ipow(t[l], e[a * d + l] - drop);
        }
        s += v;
    }
    return s;
}

static cplx cdet(int d, cplx *A)     /* Gaussian elimination, partial pivot */
{
    cplx det = 1;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (CABS(A[r * d + c]) > CABS(A[piv * d + c])) piv = r;
        if (A[piv * d + c] == 0) return 0;
        if (piv != c) {
            for (int k = 0; k < d; ++k) {
                cplx tmp = A[c * d + k];
                A[c * d + k] = A[piv * d + k];
                A[piv * d + k] = tmp;
            }
            det = -det;
        }
        det *= A[c * d + c];
        for (int r = c + 1; r < d; ++r) {
            cplx f = A[r * d + c] / A[c * d + c];
            for (int k = c; k < d; ++k) A[r * d + k] -= f * A[c * d + k];
        }
    }
    return det;
}

/* h evaluated at the real point tp (integrand without prod_{J} t^(-1+b eps)) */
static void h_series(const lims *L, const oracle_sector *s, const real *tp,
                     const real *omt, const int *inJ, double lambda,
                     series *h, int *bad_f, int *bad_u)
{
    int d = s->dim;
    cplx z[MAXD], phi[MAXD], detJ = 1;
    if (lambda > 0.0) {
        real g[MAXD];
        cplx Jm[MAXD * MAXD];
        for (int j = 0; j < d; ++j)
            g[j] = poly_d1(s->nF, s->eF, s->cF, d, tp, j);
        for (int j = 0; j < d; ++j) {
            phi[j] = 1.0 - I * lambda * omt[j] * g[j];
            z[j] = tp[j] * phi[j];
            for (int k = 0; k < d; ++k) {
                real hjk = poly_d2(s->nF, s->eF, s->cF, d, tp, j, k);
                cplx v = -I * lambda * tp[j] * omt[j] * hjk;
                if (j == k) v += 1.0 - I * lambda * (omt[j] - tp[j]) * g[j];
                Jm[j * d + k] = v;
            }
        }
        detJ = cdet(d, Jm);
    } else {
        for (int j = 0; j < d; ++j) { z[j] = tp[j]; phi[j] = 1; }
    }
    cplx Uz = poly_cplx(s->nU, s->eU, s->cU, d, z);
    cplx Fz = poly_cplx(s->nF, s->eF, s->cF, d, z);
    if (lambda > 0.0) {
        if (CIMAG(Fz) > 0) ++*bad_f;
        if (CREAL(Uz) <= 0) ++*bad_u;
    }
    cplx num = 1;
    for (int k = 0, off = 0; k < s->nP; off += s->nPt[k], ++k)
        num *= poly_cplx(s->nPt[k], s->eP + (size_t)off * d, s->cP + off, d, z);
    series f;
    s_const(h, detJ * num);
    for (int j = 0; j < d; ++j) {
        if (inJ[j]) {
            if (lambda > 0.0) {
                s_pow(L, &f, phi[j], -1.0, s->b[j]);
                s_mul(L, h, h, &f);
            }
        } else {
            s_pow(L, &f, z[j], s->a[j], s->b[j]);
            s_mul(L, h, h, &f);
        }
    }
    s_pow(L, &f, Uz, s->u0, s->u1);
    s_mul(L, h, h, &f);
    s_pow(L, &f, Fz, s->f0, s->f1);
    s_mul(L, h, h, &f);
}

/* g(t) with the subtraction of Eq. 11 for every j in J */
static void integrand(const lims *L, const oracle_sector *s, const real *t,
                      const real *omt, double lambda, series *g, int *bad_f,
                      int *bad_u)
{
    int d = s->dim, J[MAXD], nJ = 0, inJ[MAXD];
    for (int j = 0; j < d; ++j) {
        inJ[j] = (s->a[j] == -1.0);
        if (inJ[j]) J[nJ++] = j;
    }
    int ncorner = 1 << nJ;
    series *hc = malloc(sizeof(series) * ncorner);
    for (int X = 0; X < ncorner; ++X) {
        real tp[MAXD], op[MAXD];
        memcpy(tp, t, sizeof(real) * d);
        memcpy(op, omt, sizeof(real) * d);
        for (int q = 0; q < nJ; ++q)
            if (X >> q & 1) { tp[J[q]] = 0.0; op[J[q]] = 1.0; }
        h_series(L, s, tp, op, inJ, lambda, &hc[X], bad_f, bad_u);
    }
    s_zero(g);
    int full = ncorner - 1;
    for (int R = 0; R < ncorner; ++R) {
        int rest = full & ~R;
        /* inner: sum over S subset of rest of (-1)^|S| h_{R u S} */
        series inner;
        s_zero(&inner);
        for (int S = rest;; S = (S - 1) & rest) {
            int parity = __builtin_popcount(S) & 1;
            s_axpy(L, &inner, parity ? -1 : 1, &hc[R | S]);
            if (S == 0) break;
        }
        series term = inner, f;
        for (int q = 0; q < nJ; ++q) {
            int j = J[q];
            if (R >> q & 1) {
                s_div_eps(&term, &term, s->b[j]);
            } else {
                s_exp_eps(L, &f, (real)s->b[j] * RLOG(t[j]));
                for (int k = 0; k < ORD_N; ++k) f.c[k] /= t[j];
                s_mul(L, &term, &term, &f);
            }
        }
        s_axpy(L, g, 1, &term);
    }
    free(hc);
}

static void neumaier(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/*
 * Shifted lattice sums of one sector.
 *   n, z[dim]        lattice size and generating vector (Eq. 17)
 *   shifts[m][dmax]  shift vectors (Eq. 18); the sector uses the first dim
 *   r                Korobov periodiser order; lambda deformation parameter
 *   out_lo, out_len  Laurent orders returned: out_lo .. out_lo+out_len-1
 *   sums[m][out_len][2]   sum_i w g (re, im), Neumaier-compensated
 *   abss[m][out_len][2]   sum_i |w g| (re, im): scale for tolerances
 *   counts[m][3]     points with Im F(z) > 0, with Re U(z) <= 0, skipped
 * Returns 0, or -1 on bad arguments.
 */
int oracle_sector_sums(const oracle_sector *s, uint64_t n, const uint32_t *z,
                       const double *shifts, int m, int dmax, int r,
                       double lambda, int out_lo, int out_len, double *sums,
                       double *abss, int64_t *counts, int nthreads)
{
    int d = s->dim;
    if (d < 1 || d > MAXD || d > dmax || n == 0 || m < 1 || r < 0 ||
        out_lo < ORD_LO || out_lo + out_len > ORD_LO + ORD_N || out_len < 1)
        return -1;
    int nJ = 0;
    for (int j = 0; j < d; ++j) {
        if (s->a[j] == -1.0) {
            if (s->b[j] == 0.0) return -1;
            ++nJ;
        } else if (s->a[j] < -1.0) {
            return -1;
        }
    }
    int top = out_lo + out_len - 1;
    if (top + nJ >= ORD_LO + ORD_N) return -1;
    const lims L = {top + nJ, -nJ};    /* orders needed before the 1/eps divisions */

    uint64_t nchunks = (n + CHUNK - 1) / CHUNK;
    size_t slots = (size_t)m * nchunks * out_len * 2;
    double *cs = calloc(slots, sizeof(double)), *cc = calloc(slots, sizeof(double));
    double *ca = calloc(slots, sizeof(double));
    int64_t *cnt = calloc((size_t)m * nchunks * 3, sizeof(int64_t));
    if (!cs || !cc || !ca || !cnt) { free(cs); free(cc); free(ca); free(cnt); return -1; }

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t job = 0; job < (int64_t)(m * nchunks); ++job) {
        int k = (int)(job / nchunks);
        uint64_t ch = job % nchunks;
        double *S = cs + job * out_len * 2, *C = cc + job * out_len * 2;
        double *A = ca + job * out_len * 2;
        int64_t *N = cnt + job * 3;
        uint64_t i1 = (ch + 1) * CHUNK < n ? (ch + 1) * CHUNK : n;
        for (uint64_t i = ch * CHUNK; i < i1; ++i) {
            real t[MAXD], omt[MAXD];
            double w = 1.0;
            int skip = 0;
            for (int j = 0; j < d; ++j) {
                uint64_t l = (i * (uint64_t)z[j]) % n;
                double y = (double)l / (double)n + shifts[k * dmax + j];
                if (y >= 1.0) y -= 1.0;
                double tj = psi_r(y, r);
                t[j] = tj;
                omt[j] = psi_r(1.0 - y, r);    /* 1 - t by the symmetry of psi */
                w *= omega_r(y, r);
                if (tj == 0.0) skip = 1;
            }
            if (w == 0.0 || skip) { ++N[2]; continue; }
            series g;
            int bf = 0, bu = 0;
            integrand(&L, s, t, omt, lambda, &g, &bf, &bu);
            N[0] += bf != 0;
            N[1] += bu != 0;
            for (int q = 0; q < out_len; ++q) {
                cplx v = (real)w * g.c[out_lo + q - ORD_LO];
                double vr = (double)CREAL(v), vi = (double)CIMAG(v);
                neumaier(&S[2 * q], &C[2 * q], vr);
                neumaier(&S[2 * q + 1], &C[2 * q + 1], vi);
                A[2 * q] += fabs(vr);
                A[2 * q + 1] += fabs(vi);
            }
        }
    }
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < 2 * out_len; ++q) {
            double s_ = 0.0, c_ = 0.0, a_ = 0.0;
            for (uint64_t ch = 0; ch < nchunks; ++ch) {
                size_t o = ((size_t)k * nchunks + ch) * out_len * 2 + q;
                neumaier(&s_, &c_, cs[o]);
                neumaier(&s_, &c_, cc[o]);
                a_ += ca[o];
            }
            sums[(size_t)k * out_len * 2 + q] = s_ + c_;
            abss[(size_t)k * out_len * 2 + q] = a_;
        }
        for (int c = 0; c < 3; ++c) {
            int64_t tot = 0;
            for (uint64_t ch = 0; ch < nchunks; ++ch)
                tot += cnt[((size_t)k * nchunks + ch) * 3 + c];
            counts[k * 3 + c] = tot;
        }
    }
    free(cs); free(cc); free(ca); free(cnt);
    return 0;
}

/* Pointwise access for tests: the integrand series at one point t
 * (1 - t taken as computed from t). */
int oracle_point(const oracle_sector *s, const double *t, double lambda,
                 int out_lo, int out_len, double *out /* [out_len][2] */)
{
    real tt[MAXD], omt[MAXD];
    for (int j = 0; j < s->dim && j < MAXD; ++j) {
        tt[j] = t[j];
        omt[j] = 1 - (real)t[j];
    }
    int nJ = 0;
    for (int j = 0; j < s->dim; ++j) nJ += (s->a[j] == -1.0);
    int top = out_lo + out_len - 1;
    if (s->dim > MAXD || out_lo < ORD_LO || top + nJ >= ORD_LO + ORD_N) return -1;
    const lims L = {top + nJ, -nJ};
    series g;
    int bf = 0, bu = 0;
    integrand(&L, s, tt, omt, lambda, &g, &bf, &bu);
    for (int q = 0; q < out_len; ++q) {
        out[2 * q] = (double)CREAL(g.c[out_lo + q - ORD_LO]);
        out[2 * q + 1] = (double)CIMAG(g.c[out_lo + q - ORD_LO]);
    }
    return bf + 2 * bu;
}

double oracle_psi(double y, int r) { return psi_r(y, r); }
double oracle_omega(double y, int r) { return omega_r(y, r); }
