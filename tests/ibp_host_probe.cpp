// Test wrapper around the planner's host-side integration by parts
// (qmc_ibp_expand): the planned sectors' metadata and their polynomials
// evaluated at one point, in fixed-size arrays for a ctypes caller.  Built
// by tests/test_ibp_host.py into a temporary library; not part of libqmc.
#include <cstring>

#include "../paper_1508_02512_amd/csrc/qmc_internal.h"

namespace {

// sum_terms (sum_k coef[k] kin[k]) prod_v t_v^e_v
double poly_at(const std::vector<uint8_t> &e, const std::vector<double> &c, int dim, int ni,
               const double *kin, const double *t)
{
    const size_t nt = c.size() / (size_t)ni;
    double s = 0.0;
    for (size_t a = 0; a < nt; ++a) {
        double cf = 0.0;
        for (int k = 0; k < ni; ++k) cf += c[a * ni + k] * kin[k];
        double m = 1.0;
        for (int v = 0; v < dim; ++v)
            for (int p = 0; p < e[a * dim + v]; ++p) m *= t[v];
        s += cf * m;
    }
    return s;
}

} // namespace

// meta[s][6]: origin, dim, factors, coefficient window start, U terms, F terms
// expo[s][4]: u0, u1, f0, f1;  ab[s][2][8]: exponents a and b per variable
// coef[s][8][2]: C(eps);  vals[s][6]: U, F, P_1..P_4 at t_v = 0.3 + 0.1 v
extern "C" int ibp_host_expand(const qmc_problem *pb, int poles, const double *kin, int max_out,
                               int *n_out, int *meta, double *expo, double *ab, double *coef,
                               double *vals, char *err, int errlen)
{
    std::vector<qmc_ibp_sec> xs;
    const int rc = qmc_ibp_expand(pb, poles != 0, xs, err, (size_t)errlen);
    if (rc != QMC_OK) return rc;
    *n_out = (int)xs.size();
    const int ni = pb->n_inv;
    for (int s = 0; s < (int)xs.size() && s < max_out; ++s) {
        const qmc_ibp_sec &X = xs[s];
        int *m = meta + 6 * s;
        m[0] = X.origin;
        m[1] = X.dim;
        m[2] = (int)X.eP.size();
        m[3] = X.clo;
        m[4] = (int)(X.cU.size() / ni);
        m[5] = (int)(X.cF.size() / ni);
        double *x = expo + 4 * s;
        x[0] = X.u0;
        x[1] = X.u1;
        x[2] = X.f0;
        x[3] = X.f1;
        for (int v = 0; v < 8; ++v) {
            ab[16 * s + v] = v < X.dim ? X.a[v] : 0.0;
            ab[16 * s + 8 + v] = v < X.dim ? X.b[v] : 0.0;
        }
        for (int e = 0; e < 8; ++e) {
            coef[16 * s + 2 * e] = e < (int)X.C.size() ? X.C[e].real() : 0.0;
            coef[16 * s + 2 * e + 1] = e < (int)X.C.size() ? X.C[e].imag() : 0.0;
        }
        double t[8];
        for (int v = 0; v < 8; ++v) t[v] = 0.3 + 0.1 * v;
        double *y = vals + 6 * s;
        std::memset(y, 0, 6 * sizeof(double));
        y[0] = poly_at(X.eU, X.cU, X.dim, ni, kin, t);
        y[1] = poly_at(X.eF, X.cF, X.dim, ni, kin, t);
        for (size_t i = 0; i < X.eP.size() && i < 4; ++i)
            y[2 + i] = poly_at(X.eP[i], X.cP[i], X.dim, ni, kin, t);
    }
    return QMC_OK;
}
