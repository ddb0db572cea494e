// Integration by parts in the sector variables (Section II, Eq. 13).
//
// A variable with exponent alpha + beta eps, alpha < -1 (dotted
// propagators), is reduced by
//   int t^(alpha+beta eps) f dt = f(1)/(alpha+1+beta eps)
//                                 - 1/(alpha+1+beta eps) int t^(alpha+1+beta eps) df/dt dt
// until its exponent is -1 (then the subtraction of Eq. 11 takes over) or
// above -1.  In the pole mode (the paper's alternative to the subtraction)
// it is applied at -1 as well: 1/(alpha+1+beta eps) is then 1/(beta eps),
// and the sector comes out without a pole, its series C starting at
// eps^-1 per pole taken.  f = C(eps) P_1 .. P_r U^(u0+u1 eps) F^(f0+f1 eps) (times the
// other variables' monomials) stays of that form: by the product rule
// every term of df/dt either replaces a numerator factor P_i by dP_i/dt,
// or appends dU/dt (resp. dF/dt) as a factor, lowers the power of U
// (resp. F) by one and multiplies C by u0 + u1 eps (resp. f0 + f1 eps).
// Terms whose new factor vanishes identically are dropped.  The boundary
// term is the same form with the variable set to 1; a sector left without
// variables keeps one dummy variable (power 0, in no polynomial).
//
// Order of the output, fixed so that callers can match sectors one to one:
// the input sectors in order; within one, the variables in increasing
// index; each application of Eq. 13 yields the boundary term, then the
// derivative terms (numerator factors in order, then U, then F), each
// expanded completely before the next.
//
// Coefficients stay linear in the kinematic invariants (a derivative scales
// a row, setting t = 1 adds rows), so numerator factors are ordinary term
// lists for the kernels.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <map>

#include "qmc_internal.h"

namespace {

using cd = std::complex<double>;

struct wpoly {                       // sparse polynomial over the input variables
    std::vector<std::array<uint8_t, QMC_DMAX>> e;
    std::vector<double> c;           // [terms][n_inv]
};

struct wsec {
    double a[QMC_DMAX] = {}, b[QMC_DMAX] = {};
    uint32_t fixed = 0;              // variables set to 1 by a boundary term
    wpoly U, F;
    std::vector<wpoly> P;            // numerator factors
    double u0 = 0, u1 = 0, f0 = 0, f1 = 0;
    std::vector<cd> C;               // coefficient series eps^clo .. eps^(clo+NSER-1)
};

// Orders kept while expanding: every 1/(b eps) of Eq. 13 at a pole leaves
// the top order of the window incomplete, so QMC_MAX_POLES orders beyond
// the QMC_MAX_ORDERS handed out keep those exact.
constexpr int NSER = QMC_MAX_ORDERS + QMC_MAX_POLES;

struct ctx_t {
    int d = 0, ni = 0;
    bool poles = false;              // Eq. 13 at a = -1 too
    int clo = 0;                     // lowest order of the C window
    size_t produced = 0;
    char *err = nullptr;
    size_t errlen = 0;
};

constexpr size_t MAX_EXPANDED = 1u << 16;

wpoly deriv(const wpoly &p, int j, int ni)
{
    wpoly out;
    for (size_t t = 0; t < p.e.size(); ++t) {
        const int ej = p.e[t][j];
        if (ej == 0) continue;
        auto e = p.e[t];
        e[j] = (uint8_t)(ej - 1);
        out.e.push_back(e);
        for (int k = 0; k < ni; ++k) out.c.push_back(p.c[t * ni + k] * ej);
    }
    return out;
}

wpoly at_one(const wpoly &p, int j, int ni)
{
    std::map<std::array<uint8_t, QMC_DMAX>, size_t> where;
    wpoly m;
    for (size_t t = 0; t < p.e.size(); ++t) {
        auto e = p.e[t];
        e[j] = 0;
        auto it = where.find(e);
        if (it == where.end()) {
            where[e] = m.e.size();
            m.e.push_back(e);
            m.c.insert(m.c.end(), p.c.begin() + t * ni, p.c.begin() + (t + 1) * ni);
        } else {
            for (int k = 0; k < ni; ++k) m.c[it->second * ni + k] += p.c[t * ni + k];
        }
    }
    wpoly out;                       // rows that cancelled exactly are dropped
    for (size_t t = 0; t < m.e.size(); ++t) {
        bool zero = true;
        for (int k = 0; k < ni; ++k) zero &= m.c[t * ni + k] == 0.0;
        if (zero) continue;
        out.e.push_back(m.e[t]);
        out.c.insert(out.c.end(), m.c.begin() + t * ni, m.c.begin() + (t + 1) * ni);
    }
    return out;
}

// x in the C window times y = y[0] eps^ylo + y[1] eps^(ylo+1) + ..., kept in
// the window (orders above it dropped; nothing falls below it, as the
// expansion bounds the poles that Eq. 13 takes to the window's depth).
std::vector<cd> ser_mul(const std::vector<cd> &x, const std::vector<cd> &y, int ylo)
{
    std::vector<cd> r(NSER, 0.0);
    for (int p = 0; p < (int)x.size(); ++p)
        for (int q = 0; q < (int)y.size(); ++q) {
            const int i = p + q + ylo;
            if (i >= NSER) break;
            if (i >= 0) r[i] += x[p] * y[q];
        }
    return r;
}

bool ser_zero(const std::vector<cd> &x)
{
    for (const cd &v : x)
        if (v != 0.0) return false;
    return true;
}

// 1/(c0 + c1 eps) = (1/c0) sum_k (-c1/c0)^k eps^k for c0 != 0, from eps^0;
// 1/(c1 eps) for c0 = 0, from eps^-1 (ylo of the result)
std::vector<cd> ser_inv_linear(double c0, double c1, int &ylo)
{
    if (c0 == 0.0) {
        ylo = -1;
        return {1.0 / c1};
    }
    ylo = 0;
    std::vector<cd> r(NSER, 0.0);
    double v = 1.0 / c0;
    for (int k = 0; k < NSER; ++k) {
        r[k] = v;
        v *= -c1 / c0;
    }
    return r;
}

std::vector<wsec> ibp_step(const wsec &s, int j, const ctx_t &C)
{
    const double alpha = s.a[j], beta = s.b[j];
    int ilo = 0;
    const std::vector<cd> inv = ser_inv_linear(alpha + 1.0, beta, ilo);
    std::vector<wsec> out;
    {   // boundary term
        wsec t = s;
        t.fixed |= 1u << j;
        t.U = at_one(s.U, j, C.ni);
        t.F = at_one(s.F, j, C.ni);
        bool vanished = false;
        for (auto &p : t.P) {
            p = at_one(p, j, C.ni);
            vanished |= p.e.empty();
        }
        t.C = ser_mul(s.C, inv, ilo);
        if (!vanished && !ser_zero(t.C)) out.push_back(std::move(t));
    }
    std::vector<cd> minv(inv.size());
    for (size_t k = 0; k < inv.size(); ++k) minv[k] = -inv[k];
    wsec base = s;
    base.a[j] = alpha + 1.0;
    base.C = ser_mul(s.C, minv, ilo);
    for (size_t i = 0; i < s.P.size(); ++i) {
        wpoly dp = deriv(s.P[i], j, C.ni);
        if (dp.e.empty()) continue;
        wsec t = base;
        t.P[i] = std::move(dp);
        out.push_back(std::move(t));
    }
    for (int which = 0; which < 2; ++which) {
        const wpoly &Q = which == 0 ? s.U : s.F;
        const double e0 = which == 0 ? s.u0 : s.f0, e1 = which == 0 ? s.u1 : s.f1;
        wpoly dq = deriv(Q, j, C.ni);
        if (dq.e.empty() || (e0 == 0.0 && e1 == 0.0)) continue;
        wsec t = base;
        t.P.push_back(std::move(dq));
        if (which == 0) t.u0 -= 1.0;
        else t.f0 -= 1.0;
        t.C = ser_mul(base.C, std::vector<cd>{e0, e1}, 0);
        if (!ser_zero(t.C)) out.push_back(std::move(t));
    }
    return out;
}

bool expand_var(const wsec &s, int j, ctx_t &C, std::vector<wsec> &out)
{
    if ((s.fixed >> j & 1u) || s.a[j] > -1.0 || (s.a[j] == -1.0 && !C.poles)) {
        if (++C.produced > MAX_EXPANDED) return false;
        out.push_back(s);
        return true;
    }
    for (const wsec &t : ibp_step(s, j, C))
        if (!expand_var(t, j, C, out)) return false;
    return true;
}

void flatten(const wpoly &p, const std::vector<int> &keep, int ni, std::vector<uint8_t> &e,
             std::vector<double> &c)
{
    const int nd = keep.empty() ? 1 : (int)keep.size();
    e.clear();
    c.clear();
    for (size_t t = 0; t < p.e.size(); ++t) {
        for (int v = 0; v < nd; ++v) e.push_back(keep.empty() ? 0 : p.e[t][keep[v]]);
        c.insert(c.end(), p.c.begin() + t * ni, p.c.begin() + (t + 1) * ni);
    }
}

} // namespace

int qmc_ibp_expand(const qmc_problem *pb, bool poles, std::vector<qmc_ibp_sec> &out,
                   char *err, size_t errlen)
{
    out.clear();
    const int ni = pb->n_inv;
    for (int s = 0; s < pb->n_sectors; ++s) {
        const qmc_sector &S = pb->sectors[s];
        const int d = S.dim;
        ctx_t C;
        C.d = d;
        C.ni = ni;
        C.poles = poles;
        C.clo = poles ? -QMC_MAX_POLES : 0;
        if (poles) {
            // each variable with an integer power <= -1 passes -1 once, and
            // Eq. 13 there divides by b eps: at most QMC_MAX_POLES of them
            int np = 0;
            for (int j = 0; j < d; ++j) {
                const double a = S.mono_a[j];
                if (a > -1.0 || a != std::floor(a)) continue;
                if (S.mono_b[j] == 0.0) {
                    snprintf(err, errlen, "sector %d var %d: a = %g, b = 0: the pole is not "
                                          "regulated", s, j, a);
                    return QMC_EUNREGULATED;
                }
                ++np;
            }
            if (np > QMC_MAX_POLES) {
                snprintf(err, errlen, "sector %d: %d poles > %d", s, np, QMC_MAX_POLES);
                return QMC_EUNSUPPORTED;
            }
        }
        wsec w;
        for (int j = 0; j < d; ++j) {
            w.a[j] = S.mono_a[j];
            w.b[j] = S.mono_b[j];
        }
        auto load = [&](const qmc_poly &P, wpoly &q) {
            for (int t = 0; t < P.n_terms; ++t) {
                std::array<uint8_t, QMC_DMAX> e{};
                for (int j = 0; j < d; ++j) e[j] = P.exps[(size_t)t * d + j];
                q.e.push_back(e);
                q.c.insert(q.c.end(), P.coef + (size_t)t * ni, P.coef + (size_t)(t + 1) * ni);
            }
        };
        load(S.U, w.U);
        load(S.F, w.F);
        w.u0 = S.u_exp[0];
        w.u1 = S.u_exp[1];
        w.f0 = S.f_exp[0];
        w.f1 = S.f_exp[1];
        w.C.assign(NSER, 0.0);
        w.C[-C.clo] = cd(S.coef_re, S.coef_im);
        bool any = false;
        for (int j = 0; j < d; ++j) any |= w.a[j] < -1.0 || (poles && w.a[j] == -1.0);
        std::vector<wsec> cur{w};
        for (int j = 0; j < d && any; ++j) {
            std::vector<wsec> nxt;
            for (const wsec &t : cur)
                if (!expand_var(t, j, C, nxt)) {
                    snprintf(err, errlen, "sector %d: integration by parts gives more than %zu "
                                          "sectors", s, MAX_EXPANDED);
                    return QMC_EUNSUPPORTED;
                }
            cur.swap(nxt);
        }
        for (const wsec &t : cur) {
            qmc_ibp_sec x;
            x.origin = s;
            x.ibp = any;
            std::vector<int> keep;
            for (int j = 0; j < d; ++j)
                if (!(t.fixed >> j & 1u)) keep.push_back(j);
            x.dim = keep.empty() ? 1 : (int)keep.size();
            for (int v = 0; v < x.dim; ++v) {
                x.a.push_back(keep.empty() ? 0.0 : t.a[keep[v]]);
                x.b.push_back(keep.empty() ? 0.0 : t.b[keep[v]]);
            }
            flatten(t.U, keep, ni, x.eU, x.cU);
            flatten(t.F, keep, ni, x.eF, x.cF);
            for (const wpoly &p : t.P) {
                x.eP.emplace_back();
                x.cP.emplace_back();
                flatten(p, keep, ni, x.eP.back(), x.cP.back());
            }
            x.u0 = t.u0;
            x.u1 = t.u1;
            x.f0 = t.f0;
            x.f1 = t.f1;
            x.C.assign(t.C.begin(), t.C.begin() + QMC_MAX_ORDERS);
            x.clo = C.clo;
            out.push_back(std::move(x));
        }
    }
    return QMC_OK;
}
