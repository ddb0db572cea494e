// libqmc host side: context, planner, work lists, assembly of the result.
//
// The planner turns the sectors of Eq. 9 into device tables (see
// qmc_device.h); bind turns (kinematic points, lattices, shifts) into
// device inputs and a work list; run launches one integrand kernel per
// (poles, orders) class and the fixed-order reduction; fetch copies the
// per-(point, sector, shift) sums back and forms, per shift, the Laurent
// series prefactor x sum_sectors D_s S_s / n_s, then the mean over shifts
// (Eq. 19) and the error estimate (Eq. 20).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qmc.h"
#include "qmc_device.h"
#include "qmc_kernels.h"
#include "qmc_internal.h"

// ------------------------------------------------------------------ context

static int set_err(qmc_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        std::lock_guard<std::mutex> g(ctx->err_mu);
        ctx->last_error = buf;
    }
    return code;
}

int qmc_set_error(qmc_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        std::lock_guard<std::mutex> g(ctx->err_mu);
        ctx->last_error = buf;
    }
    return code;
}

#define HIP_CHECK(ctx, expr)                                                      \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess)                                                     \
            return set_err((ctx), QMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int qmc_dev_alloc(qmc_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) return QMC_OK;
    size_t used = ctx->used.load();
    if (used + bytes > ctx->budget)
        return set_err(ctx, QMC_EBUDGET, "device budget exceeded: %zu + %zu > %zu bytes",
                       used, bytes, ctx->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return set_err(ctx, QMC_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    ctx->used += bytes;
    return QMC_OK;
}

void qmc_dev_free(qmc_ctx *ctx, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    ctx->used -= bytes;
}

extern "C" int qmc_create(int device, size_t hbm_budget, int max_slots, qmc_ctx **out)
{
    if (!out) return QMC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return QMC_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return QMC_EDEVICE;
    qmc_ctx *ctx = new (std::nothrow) qmc_ctx();
    if (!ctx) return QMC_ENOMEM;
    ctx->device = device;
    ctx->budget = hbm_budget ? hbm_budget : ((size_t)64 << 30);
    ctx->max_slots = max_slots > 0 ? max_slots : 64;
    if (hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete ctx;
        return QMC_EDEVICE;
    }
    ctx->stream = ctx->own_stream;
    if (qmc_noalloc_setup(device) != QMC_OK) {
        (void)hipStreamDestroy(ctx->own_stream);
        delete ctx;
        return QMC_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->n_cu = prop.multiProcessorCount;
    *out = ctx;
    return QMC_OK;
}

extern "C" void qmc_destroy(qmc_ctx *ctx)
{
    if (!ctx) return;
    qmc_serve_shutdown(ctx);
    (void)hipSetDevice(ctx->device);
    if (ctx->own_stream) {
        (void)hipStreamSynchronize(ctx->own_stream);
        (void)hipStreamDestroy(ctx->own_stream);
    }
    delete ctx;
}

extern "C" int qmc_set_stream(qmc_ctx *ctx, void *stream)
{
    if (!ctx) return QMC_EINVAL;
    ctx->stream = stream ? (hipStream_t)stream : ctx->own_stream;
    return QMC_OK;
}

extern "C" const char *qmc_last_error(qmc_ctx *ctx)
{
    if (!ctx) return "null context";
    std::lock_guard<std::mutex> g(ctx->err_mu);
    return ctx->last_error.c_str();
}

// ------------------------------------------------------------------ planner

static uint32_t pack_exps(const uint8_t *e, const int *perm, int dim)
{
    uint32_t p = 0;
    for (int j = 0; j < dim; ++j) p |= (uint32_t)e[perm[j]] << (4 * j);
    return p;
}

// A term prod_j t_j^e_j as a product of factors taken from the per-lane
// power table of the real kernel: slot 2 j holds t_j, slot 2 j + 1 holds
// t_j^2 and slot 16 holds 1, so e_j contributes e_j / 2 factors t_j^2 and
// one t_j if e_j is odd.  Two words of four 5-bit slots (bits 5k..5k+4),
// unused slots 16; bit 30 of the first word: the second word is needed;
// bit 31: more than 8 factors (the kernel then uses exp(sum_j e_j ln t_j)).
static void term_program(uint32_t packed, uint32_t *w)
{
    uint32_t slots[8];
    int cnt = 0;
    w[0] = w[1] = 0;
    for (int j = 0; j < QMC_DMAX; ++j) {
        const uint32_t e = (packed >> (4 * j)) & 15u;
        for (uint32_t k = 0; k < e / 2 + (e & 1u); ++k) {
            if (cnt == 8) {
                w[0] = 1u << 31;
                return;
            }
            slots[cnt++] = 2u * (uint32_t)j + (k < e / 2 ? 1u : 0u);
        }
    }
    for (int k = 0; k < 8; ++k)
        w[k / 4] |= (k < cnt ? slots[k] : (uint32_t)(QMC_PROG_SLOTS - 1)) << (5 * (k % 4));
    if (cnt > 4) w[0] |= 1u << 30;
}

// Algorithmic FP64 flops of one lattice point of one sector (see DESIGN
// notes in the library documentation): add/sub/mul = 1, fma = 2, division
// and each log/exp/atan = 20.
static double sector_flops(const qmc_sec_host &h, bool deform)
{
    const double T = 20.0;
    const int d = h.dim, ks = h.ks, K = h.K;
    double f = 0.0;
    f += d * (T /*division*/ + 2 /*shift, wrap*/ + 12 /*psi, 1-psi*/ + 4 /*weight*/);
    f += d * 2;                                 // t^2, t^3
    int nlog = 0;
    for (int j = 0; j < d; ++j)
        if (j < ks || h.b[j] != 0.0 || h.aint[j] == QMC_NO_INT) ++nlog;
    f += nlog * T;
    for (const auto &nnz : h.term_nnz) f += nnz + 2;
    const int corners = 1 << ks;
    f += 2.0 * ks * (corners / 2);              // subset sums of U and F
    const double powc = h.u0i != QMC_NO_INT && h.f0i != QMC_NO_INT
                            ? std::abs(h.u0i) + std::abs(h.f0i) + (h.f0i < 0 || h.u0i < 0 ? T : 0)
                            : T;
    f += corners * (2 * T + powc + 4 + 3.0 * (K - 1));
    // numerator factors (Eq. 13): their terms are in term_nnz; one product
    // per factor in the union algebra over the 2^ks subsets (3^ks terms)
    f += h.nf * 2.0 * std::pow(3.0, ks);
    f += ks * (T + 3.0 * (K - 1));              // 1/t and (b ln t)^r / r!
    f += (corners - 1) * (K + K * (K - 1) + 3.0 * K);   // folds
    f += K * (2 + 4);                           // weight and Neumaier
    if (deform) {
        const int nd = (int)h.dterm_nnz.size();
        double dterms = 0;
        for (int v : h.dterm_nnz) dterms += v + 2;
        (void)nd;
        // per corner: derivatives, complex z and phi, Jacobian LU, complex
        // U and F (4 real flops per complex product), logs and arguments
        double per_corner = dterms + d * 8 + (4.0 * d * d * d / 3.0) * 4 +
                            4.0 * (double)h.term_nnz.size() * 3 + 2 * d * T + 4 * T;
        f += corners * per_corner + (corners - 1) * 3.0 * (K + K * (K - 1));
    }
    return f;
}

extern "C" int qmc_plan_sectors(qmc_ctx *ctx, const qmc_problem *pb,
                                const qmc_plan_opts *opts, qmc_plan **out)
{
    if (!ctx || !pb || !out) return set_err(ctx, QMC_EINVAL, "null argument");
    *out = nullptr;
    if (pb->n_sectors < 1 || !pb->sectors || pb->n_inv < 1)
        return set_err(ctx, QMC_EINVAL, "need at least one sector and n_inv >= 1");
    if (pb->eps_hi < pb->eps_lo) return set_err(ctx, QMC_EINVAL, "eps_hi < eps_lo");
    if (pb->n_pref < 1 || !pb->prefactor)
        return set_err(ctx, QMC_EINVAL, "prefactor series is empty");
    qmc_plan_opts o = {QMC_FP64, 2, 0.0, 0, QMC_POLES_SUBTRACT};
    if (opts) o = *opts;
    if (o.pole_method != QMC_POLES_SUBTRACT && o.pole_method != QMC_POLES_IBP)
        return set_err(ctx, QMC_EINVAL, "unknown pole method %d", o.pole_method);
    if (o.korobov_r < 0 || o.korobov_r > 3)
        return set_err(ctx, QMC_EUNSUPPORTED, "korobov_r must be 0..3");
    if (o.precision != QMC_FP64 && o.precision != QMC_FP32_EVAL)
        return set_err(ctx, QMC_EINVAL, "unknown precision mode %d", o.precision);
    if (!(o.lambda >= 0.0) || !std::isfinite(o.lambda))
        return set_err(ctx, QMC_EINVAL, "lambda must be finite and >= 0");

    auto *plan = new (std::nothrow) qmc_plan();
    if (!plan) return set_err(ctx, QMC_ENOMEM, "host allocation");
    static std::atomic<uint64_t> next_plan_id{1};
    plan->ctx = ctx;
    plan->id = next_plan_id++;
    plan->opts = o;
    plan->n_inv = pb->n_inv;
    plan->eps_lo = pb->eps_lo;
    plan->eps_hi = pb->eps_hi;
    plan->eps_pref_lo = pb->eps_pref_lo;
    plan->pref.assign(pb->prefactor, pb->prefactor + 2 * pb->n_pref);
    plan->n_pref = pb->n_pref;

    // inputs: dimensions and finite exponents
    for (int s = 0; s < pb->n_sectors; ++s) {
        const qmc_sector &S = pb->sectors[s];
        if (S.dim < 1 || S.dim > QMC_MAX_DIM || !S.mono_a || !S.mono_b) {
            delete plan;
            return set_err(ctx, QMC_EUNSUPPORTED, "sector %d: dim %d outside 1..%d", s, S.dim,
                           QMC_MAX_DIM);
        }
        for (int j = 0; j < S.dim; ++j)
            if (!std::isfinite(S.mono_a[j]) || !std::isfinite(S.mono_b[j])) {
                delete plan;
                return set_err(ctx, QMC_EINVAL, "sector %d: exponent not finite", s);
            }
        for (int w = 0; w < 2; ++w) {
            const qmc_poly &P = w == 0 ? S.U : S.F;
            if (P.n_terms < 1 || !P.exps || !P.coef) {
                delete plan;
                return set_err(ctx, QMC_EINVAL, "sector %d: empty polynomial", s);
            }
            for (int t = 0; t < P.n_terms * S.dim; ++t)
                if (P.exps[t] > QMC_MAX_EXP) {
                    delete plan;
                    return set_err(ctx, QMC_EUNSUPPORTED, "sector %d: exponent %d > %d", s,
                                   P.exps[t], QMC_MAX_EXP);
                }
        }
    }
    // exponents below -1: integration by parts (Eq. 13)
    std::vector<qmc_ibp_sec> xs;
    {
        char msg[256] = {};
        const int rc = qmc_ibp_expand(pb, o.pole_method == QMC_POLES_IBP, xs, msg, sizeof msg);
        if (rc != QMC_OK) {
            delete plan;
            return set_err(ctx, rc, "%s", msg);
        }
    }
    plan->n_input_sectors = pb->n_sectors;
    const int ns = (int)xs.size();
    int max_ks = 0, cmin = 0;
    // pass 1: poles and numerator factors per sector
    for (int s = 0; s < ns; ++s) {
        const qmc_ibp_sec &X = xs[s];
        if (X.ibp && o.lambda > 0.0) {
            delete plan;
            return set_err(ctx, QMC_EUNSUPPORTED,
                           "sector %d: integration by parts (%s) is supported for Euclidean "
                           "plans only (lambda = 0)", X.origin,
                           o.pole_method == QMC_POLES_IBP ? "pole method" : "exponent below -1");
        }
        if ((int)X.eP.size() > QMC_MAX_FACTORS) {
            delete plan;
            return set_err(ctx, QMC_EUNSUPPORTED,
                           "sector %d: integration by parts needs %d numerator factors > %d",
                           X.origin, (int)X.eP.size(), QMC_MAX_FACTORS);
        }
        int ks = 0;
        for (int j = 0; j < X.dim; ++j) {
            if (X.a[j] == -1.0) {
                if (X.b[j] == 0.0) {
                    delete plan;
                    return set_err(ctx, QMC_EUNREGULATED, "sector %d var %d: a = -1, b = 0",
                                   X.origin, j);
                }
                ++ks;
            }
        }
        if (ks > QMC_MAX_POLES) {
            delete plan;
            return set_err(ctx, QMC_EUNSUPPORTED, "sector %d: %d poles > %d", X.origin, ks,
                           QMC_MAX_POLES);
        }
        max_ks = std::max(max_ks, ks);
        for (size_t e = 0; e < X.C.size(); ++e)
            if (X.C[e] != 0.0) {
                cmin = std::min(cmin, X.clo + (int)e);
                break;
            }
    }
    // orders: the sum over sectors of C(eps) times the sector's series runs
    // over tot_lo .. tot_hi; a sector with ks poles carries -ks .. tot_hi - cmin
    plan->tot_hi = pb->eps_hi - pb->eps_pref_lo;
    const int kout = plan->tot_hi + 1;
    if (kout < 1 || kout > 3) {
        delete plan;
        return set_err(ctx, QMC_EUNSUPPORTED,
                       "sector orders above the poles (%d) must be 1..3", kout);
    }
    const int kb = kout - cmin;
    plan->c_lo = xs.empty() ? 0 : xs[0].clo;
    plan->tot_lo = -max_ks + cmin;
    plan->sec_lo = -max_ks;
    plan->sec_hi = plan->tot_hi - cmin;
    if (plan->sec_hi - plan->sec_lo + 1 > QMC_MAX_ORDERS ||
        plan->tot_hi - plan->tot_lo + 1 > QMC_MAX_ORDERS) {
        delete plan;
        return set_err(ctx, QMC_EUNSUPPORTED, "too many Laurent orders");
    }
    plan->kb = kb;
    plan->kstride = kb + max_ks;

    // pass 2: tables
    for (int s = 0; s < ns; ++s) {
        const qmc_ibp_sec &X = xs[s];
        qmc_sec_host h{};
        h.dim = X.dim;
        h.origin = X.origin;
        int perm[QMC_DMAX], np = 0;
        for (int j = 0; j < X.dim; ++j)
            if (X.a[j] == -1.0) perm[np++] = j;
        h.ks = np;
        for (int j = 0; j < X.dim; ++j)
            if (X.a[j] != -1.0) perm[np++] = j;
        h.K = h.ks + kb;
        h.deform = o.lambda > 0.0 ? 1 : 0;
        for (int j = 0; j < QMC_DMAX; ++j) {
            h.perm[j] = j < X.dim ? perm[j] : 0;
            h.a[j] = j < X.dim ? X.a[perm[j]] : 0.0;
            h.b[j] = j < X.dim ? X.b[perm[j]] : 0.0;
            h.aint[j] = 0;
            if (j < X.dim) {
                const double a = h.a[j];
                if (a >= 0.0 && a <= 64.0 && a == std::floor(a)) h.aint[j] = (int)a;
                else h.aint[j] = QMC_NO_INT;
            }
        }
        for (int j = 0; j < h.ks; ++j) h.inv_b[j] = 1.0 / h.b[j];
        h.u0 = X.u0;
        h.u1 = X.u1;
        h.f0 = X.f0;
        h.f1 = X.f1;
        auto as_int = [](double v) {
            return (v == std::floor(v) && std::fabs(v) <= 64.0) ? (int)v : QMC_NO_INT;
        };
        h.u0i = as_int(h.u0);
        h.f0i = as_int(h.f0);
        // terms of U, F and the numerator factors, each grouped by pole mask
        // and, within a mask, by kind (0: at most four power-table factors,
        // 1: five to eight, 2: the exp form)
        auto add_group = [&](int n_terms, const uint8_t *exps, const double *coefs,
                             int32_t *rng, int32_t *rng1, int32_t *rng2) {
            bool has_const = false;
            std::vector<std::pair<int, int>> order;   // (mask * 4 + kind, term)
            for (int a = 0; a < n_terms; ++a) {
                const uint8_t *e = exps + (size_t)a * X.dim;
                bool zero = true;
                int mask = 0;
                for (int j = 0; j < X.dim; ++j)
                    if (e[j]) zero = false;
                for (int j = 0; j < h.ks; ++j)
                    if (e[perm[j]]) mask |= 1 << j;
                has_const |= zero;
                uint32_t w[2];
                term_program(pack_exps(e, perm, X.dim), w);
                const int kind = (w[0] >> 31) ? 2 : ((w[0] >> 30) & 1u) ? 1 : 0;
                order.push_back({mask * 4 + kind, a});
            }
            std::stable_sort(order.begin(), order.end(),
                             [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                                 return x.first < y.first;
                             });
            const int32_t base = (int32_t)plan->texp.size();
            auto first_at_least = [&](int key) {
                int c = 0;
                while (c < (int)order.size() && order[c].first < key) ++c;
                return base + c;
            };
            for (int m = 0; m <= QMC_NMASK; ++m) {
                rng[m] = first_at_least(4 * m);
                if (m < QMC_NMASK) {
                    rng1[m] = first_at_least(4 * m + 1);
                    rng2[m] = first_at_least(4 * m + 2);
                }
            }
            for (auto &pr : order) {
                const uint8_t *e = exps + (size_t)pr.second * X.dim;
                plan->texp.push_back(pack_exps(e, perm, X.dim));
                uint32_t w[2];
                term_program(plan->texp.back(), w);
                if (w[0] >> 31) h.mono_log = true;
                const double *c = coefs + (size_t)pr.second * pb->n_inv;
                plan->tcoef_rows.insert(plan->tcoef_rows.end(), c, c + pb->n_inv);
                int nnz = 0;
                for (int j = 0; j < X.dim; ++j) nnz += e[j] != 0;
                h.term_nnz.push_back(nnz);
            }
            return has_const;
        };
        const int nU = (int)X.cU.size() / pb->n_inv, nF = (int)X.cF.size() / pb->n_inv;
        if (!add_group(nU, X.eU.data(), X.cU.data(), h.um, h.um1, h.um2) ||
            !add_group(nF, X.eF.data(), X.cF.data(), h.fm, h.fm1, h.fm2)) {
            delete plan;
            return set_err(ctx, QMC_EINVAL, "sector %d: U or F has no constant term%s", X.origin,
                           X.ibp ? " after integration by parts" : "");
        }
        h.nf = (int)X.eP.size();
        for (int i = 0; i < h.nf; ++i)
            add_group((int)X.cP[i].size() / pb->n_inv, X.eP[i].data(), X.cP[i].data(), h.pm[i],
                      h.pm1[i], h.pm2[i]);
        h.C = X.C;
        if (h.deform) {
            if (!qmc_cplx_supported(X.dim, h.ks, kb)) {
                delete plan;
                return set_err(ctx, QMC_EUNSUPPORTED,
                               "sector %d: deformation supports dim <= 6 with at most 2 poles "
                               "and 1-2 orders above them (dim <= 2: 1-3 orders); "
                               "got dim %d, %d poles, %d orders",
                               X.origin, X.dim, h.ks, kb);
            }
            h.lambda = o.lambda;
            // dF/dt_j and d2F/dt_j dt_k (permuted variables) as term lists
            auto add_term = [&](const uint8_t *e, const double *c, int dj, int dk, double fac) {
                uint8_t ee[QMC_DMAX] = {};
                for (int v = 0; v < X.dim; ++v) ee[v] = e[perm[v]];
                if (dj >= 0) ee[dj] -= 1;
                if (dk >= 0) ee[dk] -= 1;
                uint32_t packed = 0;
                int nnz = 0;
                for (int v = 0; v < X.dim; ++v) {
                    packed |= (uint32_t)ee[v] << (4 * v);
                    nnz += ee[v] != 0;
                }
                plan->dexp.push_back(packed);
                for (int i = 0; i < pb->n_inv; ++i) plan->dcoef_rows.push_back(fac * c[i]);
                h.dterm_nnz.push_back(nnz);
            };
            const uint8_t *Fe = X.eF.data();
            const double *Fc = X.cF.data();
            for (int j = 0; j <= QMC_DMAX; ++j) {
                h.d1[j] = (int32_t)plan->dexp.size();
                if (j >= X.dim || j == QMC_DMAX) continue;
                for (int a = 0; a < nF; ++a) {
                    const uint8_t *e = Fe + (size_t)a * X.dim;
                    const int ej = e[perm[j]];
                    if (ej > 0) add_term(e, Fc + (size_t)a * pb->n_inv, j, -1, ej);
                }
            }
            int idx = 0;
            for (int j = 0; j < QMC_DMAX; ++j)
                for (int k = j; k < QMC_DMAX; ++k, ++idx) {
                    h.d2[idx] = (int32_t)plan->dexp.size();
                    if (j >= X.dim || k >= X.dim) continue;
                    for (int a = 0; a < nF; ++a) {
                        const uint8_t *e = Fe + (size_t)a * X.dim;
                        const int ej = e[perm[j]], ek = e[perm[k]];
                        const double fac = j == k ? (double)ej * (ej - 1) : (double)ej * ek;
                        if (fac != 0.0) add_term(e, Fc + (size_t)a * pb->n_inv, j, k, fac);
                    }
                }
            h.d2[idx] = (int32_t)plan->dexp.size();
        }
        h.flops = sector_flops(h, false);
        h.flops_deform = h.deform ? sector_flops(h, true) : h.flops;
        plan->flops_per_point += h.flops;
        plan->secs.push_back(h);
    }
    plan->n_terms = (int)plan->texp.size();
    plan->max_ks = max_ks;

    // device copies of the sector headers and exponents
    std::vector<qmc_sec_dev> dev(ns);
    for (int s = 0; s < ns; ++s) dev[s] = plan->secs[s].dev();
    int rc = qmc_dev_alloc(ctx, (void **)&plan->d_sec, sizeof(qmc_sec_dev) * ns);
    if (rc == QMC_OK)
        rc = qmc_dev_alloc(ctx, (void **)&plan->d_texp, sizeof(uint32_t) * plan->texp.size());
    if (rc == QMC_OK && !plan->dexp.empty())
        rc = qmc_dev_alloc(ctx, (void **)&plan->d_dexp, sizeof(uint32_t) * plan->dexp.size());
    std::vector<double> texpd(plan->texp.size() * QMC_DMAX);
    std::vector<uint32_t> tprog(plan->texp.size() * 2);
    for (size_t t = 0; t < plan->texp.size(); ++t) {
        for (int j = 0; j < QMC_DMAX; ++j)
            texpd[t * QMC_DMAX + j] = (double)((plan->texp[t] >> (4 * j)) & 15u);
        term_program(plan->texp[t], &tprog[2 * t]);
    }
    if (rc == QMC_OK)
        rc = qmc_dev_alloc(ctx, (void **)&plan->d_texpd, sizeof(double) * texpd.size());
    if (rc == QMC_OK)
        rc = qmc_dev_alloc(ctx, (void **)&plan->d_tprog, sizeof(uint32_t) * tprog.size());
    // every factor of a term as the byte offset of its power-table slot in
    // a lane's column (slot stride QMC_BLOCK elements of the plan's type)
    const uint32_t esize = o.precision == QMC_FP32_EVAL ? 4u : 8u;
    // first all terms' factors 1-4, then all terms' factors 5-8
    const size_t nterm = plan->texp.size();
    std::vector<uint32_t> toff(nterm * 8);
    for (size_t t = 0; t < nterm; ++t)
        for (int k = 0; k < 8; ++k) {
            const uint32_t slot = (tprog[2 * t + k / 4] >> (5 * (k % 4))) & 31u;
            toff[(k / 4) * nterm * 4 + 4 * t + (k % 4)] = slot * QMC_BLOCK * esize;
        }
    if (rc == QMC_OK)
        rc = qmc_dev_alloc(ctx, (void **)&plan->d_toff, sizeof(uint32_t) * toff.size());
    std::vector<uint32_t> dprog(plan->dexp.size() * 2);
    for (size_t t = 0; t < plan->dexp.size(); ++t) term_program(plan->dexp[t], &dprog[2 * t]);
    if (rc == QMC_OK && !dprog.empty())
        rc = qmc_dev_alloc(ctx, (void **)&plan->d_dprog, sizeof(uint32_t) * dprog.size());
    if (rc != QMC_OK) {
        qmc_plan_free(plan);
        return rc;
    }
    hipError_t e = hipMemcpy(plan->d_sec, dev.data(), sizeof(qmc_sec_dev) * ns,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(plan->d_texp, plan->texp.data(), sizeof(uint32_t) * plan->texp.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !plan->dexp.empty())
        e = hipMemcpy(plan->d_dexp, plan->dexp.data(), sizeof(uint32_t) * plan->dexp.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(plan->d_texpd, texpd.data(), sizeof(double) * texpd.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(plan->d_tprog, tprog.data(), sizeof(uint32_t) * tprog.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !dprog.empty())
        e = hipMemcpy(plan->d_dprog, dprog.data(), sizeof(uint32_t) * dprog.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(plan->d_toff, toff.data(), sizeof(uint32_t) * toff.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        qmc_plan_free(plan);
        return set_err(ctx, QMC_EDEVICE, "upload: %s", hipGetErrorString(e));
    }
    *out = plan;
    return QMC_OK;
}

qmc_sec_dev qmc_sec_host::dev() const
{
    qmc_sec_dev d{};
    d.dim = dim;
    d.ks = ks;
    d.K = K;
    d.deform = deform;
    for (int j = 0; j < QMC_DMAX; ++j) {
        d.perm[j] = perm[j];
        d.a[j] = a[j];
        d.b[j] = b[j];
        d.inv_b[j] = inv_b[j];
        d.aint[j] = aint[j];
    }
    for (int m = 0; m <= QMC_NMASK; ++m) {
        d.um[m] = um[m];
        d.fm[m] = fm[m];
    }
    for (int m = 0; m < QMC_NMASK; ++m) {
        d.um1[m] = um1[m];
        d.um2[m] = um2[m];
        d.fm1[m] = fm1[m];
        d.fm2[m] = fm2[m];
    }
    for (int j = 0; j <= QMC_DMAX; ++j) d.d1[j] = d1[j];
    for (int j = 0; j <= QMC_DMAX * (QMC_DMAX + 1) / 2; ++j) d.d2[j] = d2[j];
    d.u0 = u0;
    d.u1 = u1;
    d.f0 = f0;
    d.f1 = f1;
    d.u0i = u0i;
    d.f0i = f0i;
    d.lambda = lambda;
    // ln t_j feeds the pole variables, t_j^(b_j eps), non-integer powers
    // t_j^a_j and the exp-form monomials; the others skip it
    d.lnmask = 0;
    for (int j = 0; j < dim; ++j)
        if (mono_log || j < ks || b[j] != 0.0 || aint[j] == QMC_NO_INT) d.lnmask |= 1 << j;
    d.nf = nf;
    for (int i = 0; i < QMC_NFMAX; ++i) {
        for (int m = 0; m <= QMC_NMASK; ++m) d.pm[i][m] = pm[i][m];
        for (int m = 0; m < QMC_NMASK; ++m) {
            d.pm1[i][m] = pm1[i][m];
            d.pm2[i][m] = pm2[i][m];
        }
    }
    return d;
}

extern "C" void qmc_plan_free(qmc_plan *plan)
{
    if (!plan) return;
    qmc_ctx *ctx = plan->ctx;
    {
        // the autotuner's choices for this plan go with it
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        const std::string prefix = std::to_string((unsigned long long)plan->id) + "/";
        for (auto it = ctx->tuned.begin(); it != ctx->tuned.end();)
            it = it->first.compare(0, prefix.size(), prefix) == 0 ? ctx->tuned.erase(it)
                                                                  : std::next(it);
    }
    qmc_dev_free(ctx, plan->d_sec, sizeof(qmc_sec_dev) * plan->secs.size());
    qmc_dev_free(ctx, plan->d_texp, sizeof(uint32_t) * plan->texp.size());
    qmc_dev_free(ctx, plan->d_texpd, sizeof(double) * plan->texp.size() * QMC_DMAX);
    qmc_dev_free(ctx, plan->d_tprog, sizeof(uint32_t) * plan->texp.size() * 2);
    qmc_dev_free(ctx, plan->d_toff, sizeof(uint32_t) * plan->texp.size() * 8);
    qmc_dev_free(ctx, plan->d_dprog, sizeof(uint32_t) * plan->dexp.size() * 2);
    qmc_dev_free(ctx, plan->d_dexp, sizeof(uint32_t) * plan->dexp.size());
    delete plan;
}

extern "C" int qmc_plan_get_info(const qmc_plan *plan, qmc_plan_info *info)
{
    if (!plan || !info) return QMC_EINVAL;
    info->n_sectors = (int32_t)plan->secs.size();
    info->n_inv = plan->n_inv;
    info->sec_lo = plan->sec_lo;
    info->sec_orders = plan->sec_hi - plan->sec_lo + 1;
    info->eps_lo = plan->eps_lo;
    info->eps_hi = plan->eps_hi;
    info->max_poles = plan->max_ks;
    info->deform = plan->opts.lambda > 0.0;
    info->flops_per_point = plan->flops_per_point;
    info->n_input_sectors = plan->n_input_sectors;
    int nf = 0;
    for (const qmc_sec_host &h : plan->secs) nf = std::max(nf, h.nf);
    info->max_factors = nf;
    return QMC_OK;
}

extern "C" int qmc_plan_sector_info(const qmc_plan *plan, int32_t s, qmc_sector_info *out)
{
    if (!plan || !out || s < 0 || s >= (int32_t)plan->secs.size()) return QMC_EINVAL;
    const qmc_sec_host &h = plan->secs[s];
    *out = qmc_sector_info{};
    out->origin = h.origin;
    out->dim = h.dim;
    out->poles = h.ks;
    out->factors = h.nf;
    out->u_exp[0] = h.u0;
    out->u_exp[1] = h.u1;
    out->f_exp[0] = h.f0;
    out->f_exp[1] = h.f1;
    for (size_t e = 0; e < h.C.size() && e < (size_t)QMC_MAX_ORDERS; ++e) {
        out->coef[e][0] = h.C[e].real();
        out->coef[e][1] = h.C[e].imag();
    }
    out->coef_lo = plan->c_lo;
    return QMC_OK;
}

// ------------------------------------------------------------------ jobs

void qmc_contract(const qmc_plan *plan, const double *kin, double *coef, double *dcoef)
{
    const int ni = plan->n_inv;
    for (int t = 0; t < plan->n_terms; ++t) {
        const double *row = plan->tcoef_rows.data() + (size_t)t * ni;
        double c = 0.0;
        for (int i = 0; i < ni; ++i) c += row[i] * kin[i];
        coef[t] = c;
    }
    const int nd = (int)plan->dexp.size();
    for (int t = 0; t < nd; ++t) {
        const double *row = plan->dcoef_rows.data() + (size_t)t * ni;
        double c = 0.0;
        for (int i = 0; i < ni; ++i) c += row[i] * kin[i];
        dcoef[t] = c;
    }
}

// A sector is deformed at a kinematic point only if some coefficient of its
// F is negative there; with all coefficients >= 0 (and the constant term
// > 0) F is positive on the whole cube and the real kernel applies.  The
// deformation parameter is made dimensionless by the largest |coefficient|
// of the sector's F at that point: lambda_eff = lambda / max |c|.
// Returns the complex kernel width (0 for the real kernel).
int qmc_sector_mode(const qmc_plan *plan, int s, const double *coef, double *lam)
{
    const qmc_sec_host &h = plan->secs[s];
    *lam = 0.0;
    if (!h.deform) return 0;
    bool deform = false;
    double cmax = 0.0;
    for (int q = h.fm[0]; q < h.fm[QMC_NMASK]; ++q) {
        deform |= coef[q] < 0.0;
        cmax = std::max(cmax, std::fabs(coef[q]));
    }
    if (!deform) return 0;
    *lam = plan->opts.lambda / cmax;
    return qmc_cplx_dm(h.dim);
}

int qmc_class_grid(const qmc_class &c)
{
    const int items = c.end - c.begin;
    const int grid = c.grid > 0 ? std::min(c.grid, items) : items;
    // a launch may hold fewer than 2^32 work-items in total; the kernels
    // loop over the items with stride gridDim, so a capped grid still
    // covers every item
    return std::min(grid, QMC_MAX_GRID);
}

hipError_t qmc_launch_class(const qmc_plan *plan, const qmc_class &c, const qmc_launch_args &A,
                            hipStream_t stream)
{
    const int grid = qmc_class_grid(c);
    const bool fp32 = plan->opts.precision == QMC_FP32_EVAL;
    if (c.deform) return qmc_launch_cplx(c.dm, c.ks, c.kb, fp32, c.variant, A, grid, stream);
    return qmc_launch_real(c.ks, c.kb, fp32, c.variant, c.num != 0, A, grid, stream);
}

void qmc_job_release(qmc_job *job)
{
    if (!job) return;
    qmc_ctx *ctx = job->ctx;
    for (auto &b : job->bufs) qmc_dev_free(ctx, b.first, b.second);
    job->bufs.clear();
    if (job->ev0) (void)hipEventDestroy(job->ev0);
    if (job->ev1) (void)hipEventDestroy(job->ev1);
    job->ev0 = job->ev1 = nullptr;
    for (hipEvent_t e : job->ev_cls) (void)hipEventDestroy(e);
    job->ev_cls.clear();
    if (job->graph) (void)hipGraphExecDestroy(job->graph);
    job->graph = nullptr;
    if (job->h_out) (void)hipHostFree(job->h_out);
    if (job->h_gviol) (void)hipHostFree(job->h_gviol);
    job->h_out = nullptr;
    job->h_gviol = nullptr;
}

std::string qmc_tune_key(const qmc_plan *plan, int ks, int dm, int num, uint64_t n)
{
    int lg = 0;
    while ((2ull << lg) <= n) ++lg;
    char buf[128];
    // keyed by the plan's id, never its address: a freed plan's address
    // can be reused by a later, different plan
    snprintf(buf, sizeof buf, "%llu/%d/%d/%d/%d/%d", (unsigned long long)plan->id, ks, dm, num,
             plan->opts.precision, lg);
    return buf;
}

template <class T>
static int job_upload(qmc_job *job, T **dptr, const T *src, size_t count)
{
    size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
    int rc = qmc_dev_alloc(job->ctx, (void **)dptr, bytes);
    if (rc != QMC_OK) return rc;
    job->bufs.push_back({(void *)*dptr, bytes});
    if (count && src) {
        hipError_t e = hipMemcpyAsync(*dptr, src, sizeof(T) * count, hipMemcpyHostToDevice,
                                      job->ctx->stream);
        if (e != hipSuccess)
            return set_err(job->ctx, QMC_EDEVICE, "upload: %s", hipGetErrorString(e));
    }
    return QMC_OK;
}

// The host side of a bind: validates the inputs and fills the job's
// classes, sizes and the host arrays of its device inputs (no device work).
int qmc_job_prepare(qmc_ctx *ctx, const qmc_plan *plan, const double *kin, int32_t n_points,
                    const qmc_lattice *lat, const qmc_lattice *lat_per_sector,
                    const double *shifts, int32_t m, int ppl_override, int grid_override,
                    qmc_job *job, qmc_job_host &H)
{
    if (!ctx || !plan || !kin || !shifts) return set_err(ctx, QMC_EINVAL, "null argument");
    if (n_points < 1) return set_err(ctx, QMC_EINVAL, "n_points < 1");
    if (m < 2) return set_err(ctx, QMC_EINVAL, "need m >= 2 shifts for the error estimate");
    if (!lat && !lat_per_sector) return set_err(ctx, QMC_EINVAL, "no lattice given");
    const int ns = (int)plan->secs.size();
    job->ctx = ctx;
    job->plan = plan;
    job->n_points = n_points;
    job->m = m;

    // lattices per sector, components permuted like the sector's variables
    std::vector<qmc_lat_dev> &lats = H.lats;
    lats.assign(ns, qmc_lat_dev{});
    job->n_per_sector.resize(ns);
    for (int s = 0; s < ns; ++s) {
        const qmc_lattice &L = lat_per_sector ? lat_per_sector[s] : *lat;
        if (L.n < 2 || L.n >= (1ull << 31) || !L.z)
            return set_err(ctx, QMC_EINVAL, "sector %d: lattice size %llu outside [2, 2^31)", s,
                           (unsigned long long)L.n);
        const qmc_sec_host &h = plan->secs[s];
        qmc_lat_dev d{};
        d.n = (uint32_t)L.n;
        d.inv_n = 1.0 / (double)L.n;
        for (int j = 0; j < QMC_DMAX; ++j)
            d.z[j] = j < h.dim ? (uint32_t)(L.z[h.perm[j]] % L.n) : 0u;
        lats[s] = d;
        job->n_per_sector[s] = L.n;
    }
    // coefficients contracted with the kinematics of every point
    const int nt = plan->n_terms, ni = plan->n_inv;
    const int nd = (int)plan->dexp.size();
    std::vector<double> &coef = H.coef, &dcoef = H.dcoef;
    coef.assign((size_t)n_points * nt, 0.0);
    dcoef.assign((size_t)n_points * nd, 0.0);
    for (int p = 0; p < n_points; ++p)
        qmc_contract(plan, kin + (size_t)p * ni, coef.data() + (size_t)p * nt,
                     dcoef.data() + (size_t)p * nd);
    // work list: class-major (poles, kernel width), then point, sector, shift, tile
    uint64_t total = 0;
    for (int s = 0; s < ns; ++s) total += job->n_per_sector[s];
    total *= (uint64_t)m * n_points;
    int ppl = ppl_override > 0 ? ppl_override : plan->opts.points_per_lane;
    if (ppl <= 0) {
        const uint64_t target_items = 1ull << 17;
        uint64_t want = (total + (uint64_t)QMC_BLOCK * target_items - 1) /
                        ((uint64_t)QMC_BLOCK * target_items);
        ppl = (int)std::min<uint64_t>(std::max<uint64_t>(want, 4), 1 << 14);
    }
    job->ppl = ppl;
    uint64_t nmax_sec = 0;
    for (int s = 0; s < ns; ++s) nmax_sec = std::max<uint64_t>(nmax_sec, job->n_per_sector[s]);
    const int n_groups = n_points * ns * m;
    std::vector<int32_t> &gbeg = H.gbeg, &gend = H.gend;
    gbeg.assign(n_groups, 0);
    gend.assign(n_groups, 0);
    std::vector<qmc_item> &items = H.items;
    items.clear();
    std::vector<int> key_of((size_t)n_points * ns);
    std::vector<double> &lam = H.lam;
    lam.assign((size_t)n_points * ns, 0.0);
    // (ks, dm or 0 for real, numerator factors or not) of every class
    std::vector<std::array<int, 3>> keys;
    for (int p = 0; p < n_points; ++p)
        for (int s = 0; s < ns; ++s) {
            const int dm = qmc_sector_mode(plan, s, coef.data() + (size_t)p * nt,
                                           &lam[(size_t)p * ns + s]);
            const std::array<int, 3> key{plan->secs[s].ks, dm, qmc_num_class(plan, s)};
            auto it = std::find(keys.begin(), keys.end(), key);
            if (it == keys.end()) {
                keys.push_back(key);
                it = keys.end() - 1;
            }
            key_of[(size_t)p * ns + s] = (int)(it - keys.begin());
        }
    std::vector<int> order(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return keys[x] < keys[y]; });
    for (int ki : order) {
        qmc_class c{};
        c.ks = keys[ki][0];
        c.dm = keys[ki][1];
        c.num = keys[ki][2];
        c.deform = c.dm != 0;
        c.kb = plan->kb;
        c.begin = (int)items.size();
        c.ppl = ppl;
        c.grid = grid_override > 0 ? grid_override * ctx->n_cu : 0;
        if (ppl_override <= 0 && plan->opts.points_per_lane <= 0) {
            std::lock_guard<std::mutex> g(ctx->tune_mu);
            auto t = ctx->tuned.find(qmc_tune_key(plan, c.ks, c.dm, c.num, nmax_sec));
            if (t != ctx->tuned.end()) {
                c.ppl = t->second.ppl;
                c.grid = t->second.grid_per_cu * ctx->n_cu;
                c.variant = t->second.variant;
            }
        }
        const uint64_t tile = (uint64_t)QMC_BLOCK * c.ppl;
        for (int p = 0; p < n_points; ++p)
            for (int s = 0; s < ns; ++s) {
                if (key_of[(size_t)p * ns + s] != ki) continue;
                const uint64_t n = job->n_per_sector[s];
                for (int k = 0; k < m; ++k) {
                    const int g = (p * ns + s) * m + k;
                    gbeg[g] = (int32_t)items.size();
                    for (uint64_t st = 0; st < n; st += tile) {
                        qmc_item it{};
                        it.sector = s;
                        it.point = p;
                        it.shift = k;
                        it.group = g;
                        it.lat = s;
                        it.start = (uint32_t)st;
                        it.count = (uint32_t)std::min<uint64_t>(tile, n - st);
                        it.stride = 1;
                        items.push_back(it);
                        c.evals += it.count;
                        c.flops += it.count * (c.dm ? plan->secs[s].flops_deform
                                                    : plan->secs[s].flops);
                    }
                    gend[g] = (int32_t)items.size();
                }
            }
        c.end = (int)items.size();
        if (c.end > c.begin) job->classes.push_back(c);
    }
    if (items.size() > (size_t)INT32_MAX) return set_err(ctx, QMC_EINVAL, "work list too long");
    job->n_items = (int)items.size();
    job->n_groups = n_groups;
    job->evals = total;
    job->h_out_n = (size_t)n_groups * plan->kstride * 2;
    H.shifts = shifts;
    return QMC_OK;
}

int qmc_bind_impl(qmc_ctx *ctx, const qmc_plan *plan, const double *kin, int32_t n_points,
                  const qmc_lattice *lat, const qmc_lattice *lat_per_sector,
                  const double *shifts, int32_t m, int ppl_override, int grid_override,
                  bool class_timing, qmc_job **out)
{
    if (!out) return set_err(ctx, QMC_EINVAL, "null argument");
    *out = nullptr;
    auto *job = new (std::nothrow) qmc_job();
    if (!job) return set_err(ctx, QMC_ENOMEM, "host allocation");
    qmc_job_host H;
    int rc = qmc_job_prepare(ctx, plan, kin, n_points, lat, lat_per_sector, shifts, m,
                             ppl_override, grid_override, job, H);
    if (rc) {
        delete job;
        return rc;
    }
    (void)hipSetDevice(ctx->device);
    const int n_groups = job->n_groups;
    if (!rc) rc = job_upload(job, &job->d_lat, H.lats.data(), H.lats.size());
    if (!rc) rc = job_upload(job, &job->d_coef, H.coef.data(), H.coef.size());
    if (!rc) rc = job_upload(job, &job->d_dcoef, H.dcoef.data(), H.dcoef.size());
    if (!rc) rc = job_upload(job, &job->d_lam, H.lam.data(), H.lam.size());
    if (!rc) rc = job_upload(job, &job->d_shift, shifts, (size_t)m * QMC_DMAX);
    if (!rc) rc = job_upload(job, &job->d_items, H.items.data(), H.items.size());
    if (!rc) rc = job_upload(job, &job->d_gbeg, H.gbeg.data(), H.gbeg.size());
    if (!rc) rc = job_upload(job, &job->d_gend, H.gend.data(), H.gend.size());
    if (!rc)
        rc = job_upload<double>(job, &job->d_partial, nullptr,
                                (size_t)job->n_items * plan->kstride * 4);
    if (!rc) rc = job_upload<int32_t>(job, &job->d_viol, nullptr, (size_t)job->n_items);
    if (!rc)
        rc = job_upload<double>(job, &job->d_out, nullptr, (size_t)n_groups * plan->kstride * 2);
    if (!rc) rc = job_upload<int32_t>(job, &job->d_gviol, nullptr, (size_t)n_groups);
    // the uploads read the host arrays of H, which end with this call
    if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = set_err(ctx, QMC_EDEVICE, "upload failed");
    if (!rc && (hipEventCreate(&job->ev0) != hipSuccess || hipEventCreate(&job->ev1) != hipSuccess))
        rc = set_err(ctx, QMC_EDEVICE, "hipEventCreate failed");
    if (rc) {
        qmc_job_release(job);
        delete job;
        return rc;
    }
    if (hipHostMalloc((void **)&job->h_out, sizeof(double) * job->h_out_n) != hipSuccess ||
        hipHostMalloc((void **)&job->h_gviol, sizeof(int32_t) * n_groups) != hipSuccess) {
        qmc_job_release(job);
        delete job;
        return set_err(ctx, QMC_ENOMEM, "pinned host allocation");
    }
    if (class_timing) {
        job->ev_cls.resize(job->classes.size() + 1);
        for (auto &e : job->ev_cls) (void)hipEventCreate(&e);
    }
    *out = job;
    return QMC_OK;
}

extern "C" int qmc_bind(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                        int32_t n_points, const qmc_lattice *lat,
                        const qmc_lattice *lat_per_sector, const double *shifts, int32_t m,
                        qmc_job **out)
{
    return qmc_bind_impl(ctx, plan, kin, n_points, lat, lat_per_sector, shifts, m, 0, 0, false,
                         out);
}

// The launch sequence of a bound job on the context stream: one integrand
// launch per class (bracketed by the class events when timing), the
// fixed-order reduction and the copies of the group sums and violation
// counts into job->h_out and job->h_gviol.
hipError_t qmc_enqueue(qmc_job *job, bool timing)
{
    qmc_ctx *ctx = job->ctx;
    const qmc_plan *plan = job->plan;
    qmc_launch_args A{};
    A.sec = plan->d_sec;
    A.lat = job->d_lat;
    A.texp = plan->d_texp;
    A.texpd = plan->d_texpd;
    A.tprog = plan->d_tprog;
    A.toff = plan->d_toff;
    A.dprog = plan->d_dprog;
    A.tcoef = job->d_coef;
    A.dexp = plan->d_dexp;
    A.dcoef = job->d_dcoef;
    A.shifts = job->d_shift;
    A.lam = job->d_lam;
    A.n_sec = (int32_t)plan->secs.size();
    A.items = job->d_items;
    A.partial = job->d_partial;
    A.viol = job->d_viol;
    A.n_terms = plan->n_terms;
    A.n_dterms = (int32_t)plan->dexp.size();
    A.kstride = plan->kstride;
    A.korobov_r = plan->opts.korobov_r;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < job->classes.size() && e == hipSuccess; ++i) {
        const qmc_class &c = job->classes[i];
        if (timing && !job->ev_cls.empty()) e = hipEventRecord(job->ev_cls[i], ctx->stream);
        A.item_begin = c.begin;
        A.item_end = c.end;
        if (e == hipSuccess) e = qmc_launch_class(plan, c, A, ctx->stream);
    }
    if (e == hipSuccess && timing && !job->ev_cls.empty())
        e = hipEventRecord(job->ev_cls.back(), ctx->stream);
    if (e == hipSuccess && timing && job->ev1) e = hipEventRecord(job->ev1, ctx->stream);
    if (e == hipSuccess)
        e = qmc_launch_reduce(job->d_partial, job->d_viol, job->d_gbeg, job->d_gend,
                              job->n_groups, plan->kstride, job->d_out, job->d_gviol,
                              ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(job->h_out, job->d_out, sizeof(double) * job->h_out_n,
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(job->h_gviol, job->d_gviol, sizeof(int32_t) * job->n_groups,
                           hipMemcpyDeviceToHost, ctx->stream);
    return e;
}

extern "C" int qmc_run(qmc_job *job)
{
    if (!job) return QMC_EINVAL;
    qmc_ctx *ctx = job->ctx;
    (void)hipSetDevice(ctx->device);
    auto enqueue = [&](bool timing) { return qmc_enqueue(job, timing); };
    if (job->use_graph) {
        // the whole sequence as one graph, captured once and replayed
        if (!job->graph) {
            hipGraph_t g = nullptr;
            HIP_CHECK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue(false);
            const hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
            HIP_CHECK(ctx, e);
            HIP_CHECK(ctx, e2);
            const hipError_t e3 = hipGraphInstantiate(&job->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_CHECK(ctx, e3);
        }
        HIP_CHECK(ctx, hipEventRecord(job->ev0, ctx->stream));
        HIP_CHECK(ctx, hipGraphLaunch(job->graph, ctx->stream));
        HIP_CHECK(ctx, hipEventRecord(job->ev1, ctx->stream));
    } else {
        // ev0 .. ev1 brackets the integrand kernels only
        HIP_CHECK(ctx, hipEventRecord(job->ev0, ctx->stream));
        HIP_CHECK(ctx, enqueue(true));
    }
    job->cls_timed = !job->use_graph && !job->ev_cls.empty();
    job->launched = true;
    return QMC_OK;
}

// Laurent assembly and statistics (Eqs. 19-20) from the per-group sums.
int qmc_assemble(const qmc_plan *plan, int n_points, int m, const std::vector<uint64_t> &nsec,
                 const double *gsum /* [groups][kstride][2] */, qmc_result *out)
{
    const int ns = (int)plan->secs.size();
    const int K = plan->tot_hi - plan->tot_lo + 1;
    const int no = plan->eps_hi - plan->eps_lo + 1;
    std::vector<std::complex<double>> tot(K), Q((size_t)m * no);
    for (int p = 0; p < n_points; ++p) {
        for (int k = 0; k < m; ++k) {
            std::fill(tot.begin(), tot.end(), 0.0);
            for (int s = 0; s < ns; ++s) {
                const qmc_sec_host &h = plan->secs[s];
                const double *g = gsum + ((size_t)((p * ns + s) * m + k)) * plan->kstride * 2;
                for (int q = 0; q < h.K; ++q) {
                    const int order = q - h.ks;
                    const std::complex<double> v(g[2 * q], g[2 * q + 1]);
                    // the sector's coefficient series C(eps) (D, or Eq. 13's)
                    for (size_t e = 0; e < h.C.size(); ++e) {
                        const int j = order + plan->c_lo + (int)e - plan->tot_lo;
                        if (j >= K) break;
                        if (j >= 0 && h.C[e] != 0.0) tot[j] += h.C[e] * v / (double)nsec[s];
                    }
                }
            }
            for (int oi = 0; oi < no; ++oi) {
                const int order = plan->eps_lo + oi;
                std::complex<double> acc = 0.0;
                for (int j = 0; j < K; ++j) {
                    const int pp = order - (plan->tot_lo + j) - plan->eps_pref_lo;
                    if (pp < 0 || pp >= plan->n_pref) continue;
                    acc += std::complex<double>(plan->pref[2 * pp], plan->pref[2 * pp + 1]) * tot[j];
                }
                Q[(size_t)k * no + oi] = acc;
            }
        }
        for (int oi = 0; oi < no; ++oi) {
            double mr = 0.0, mi = 0.0;
            for (int k = 0; k < m; ++k) {
                mr += Q[(size_t)k * no + oi].real();
                mi += Q[(size_t)k * no + oi].imag();
            }
            mr /= m;
            mi /= m;
            double vr = 0.0, vi = 0.0;
            for (int k = 0; k < m; ++k) {
                const double dr = Q[(size_t)k * no + oi].real() - mr;
                const double di = Q[(size_t)k * no + oi].imag() - mi;
                vr += dr * dr;
                vi += di * di;
            }
            qmc_coeff &c = out->coeff[(size_t)p * no + oi];
            c.re = mr;
            c.im = mi;
            c.err_re = std::sqrt(vr / ((double)m * (m - 1)));
            c.err_im = std::sqrt(vi / ((double)m * (m - 1)));
        }
        if (out->per_shift)
            for (int k = 0; k < m; ++k)
                for (int oi = 0; oi < no; ++oi) {
                    double *d = out->per_shift + (((size_t)p * m + k) * no + oi) * 2;
                    d[0] = Q[(size_t)k * no + oi].real();
                    d[1] = Q[(size_t)k * no + oi].imag();
                }
    }
    if (out->sector_sums) {
        const int K2 = K;
        for (int p = 0; p < n_points; ++p)
            for (int s = 0; s < ns; ++s)
                for (int k = 0; k < m; ++k) {
                    const qmc_sec_host &h = plan->secs[s];
                    const double *g = gsum + ((size_t)((p * ns + s) * m + k)) * plan->kstride * 2;
                    double *d = out->sector_sums + (((size_t)(p * ns + s) * m + k) * K2) * 2;
                    for (int j = 0; j < K2 * 2; ++j) d[j] = 0.0;
                    for (int q = 0; q < h.K; ++q) {
                        const int j = q - h.ks - plan->sec_lo;
                        d[2 * j] = g[2 * q];
                        d[2 * j + 1] = g[2 * q + 1];
                    }
                }
    }
    return QMC_OK;
}

extern "C" int qmc_fetch(qmc_job *job, qmc_result *out)
{
    if (!job || !out || !out->coeff) return QMC_EINVAL;
    qmc_ctx *ctx = job->ctx;
    if (!job->launched) return set_err(ctx, QMC_EINVAL, "qmc_fetch before qmc_run");
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.0f;
    HIP_CHECK(ctx, hipEventElapsedTime(&ms, job->ev0, job->ev1));
    job->launched = false;
    out->kernel_ms = ms;
    job->cls_ms.assign(job->classes.size(), -1.0);
    if (job->cls_timed)
        for (size_t i = 0; i < job->classes.size(); ++i) {
            float cms = 0.0f;
            if (hipEventElapsedTime(&cms, job->ev_cls[i], job->ev_cls[i + 1]) == hipSuccess)
                job->cls_ms[i] = cms;
        }
    return qmc_result_fill(job, job->h_out, job->h_gviol, out);
}

// Assembly (Eqs. 19-20) and the counters of a finished run from its group
// sums and per-group violation counts (host memory).
int qmc_result_fill(qmc_job *job, const double *gsum, const int32_t *gviol, qmc_result *out)
{
    qmc_assemble(job->plan, job->n_points, job->m, job->n_per_sector, gsum, out);
    long viol = 0;
    for (int i = 0; i < job->n_groups; ++i) viol += gviol[i];
    out->evals = job->evals;
    out->n_final = job->n_per_sector.empty() ? 0 : job->n_per_sector[0];
    out->deform_violations = (int32_t)std::min<long>(viol, INT32_MAX);
    out->status = viol ? QMC_EDEFORM : QMC_OK;
    double fl = 0.0;
    for (const qmc_class &c : job->classes) fl += c.flops;
    out->algo_flops = fl;
    return out->status == QMC_OK
               ? QMC_OK
               : set_err(job->ctx, out->status, "%ld points violated the sign conditions", viol);
}

extern "C" void qmc_job_free(qmc_job *job)
{
    if (!job) return;
    if (job->launched) (void)hipStreamSynchronize(job->ctx->stream);
    qmc_job_release(job);
    delete job;
}

extern "C" int qmc_integrate(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                             int32_t n_points, const qmc_lattice *lat,
                             const qmc_lattice *lat_per_sector, const double *shifts,
                             int32_t m, qmc_result *out)
{
    if (!out || !out->coeff) return set_err(ctx, QMC_EINVAL, "null result");
    qmc_job *job = nullptr;
    int rc = qmc_bind(ctx, plan, kin, n_points, lat, lat_per_sector, shifts, m, &job);
    if (rc) return rc;
    rc = qmc_run(job);
    if (!rc) rc = qmc_fetch(job, out);
    qmc_job_free(job);
    return rc;
}

extern "C" int qmc_size_lattices(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                                 const qmc_lattice *pilot, const double *shifts, int32_t m,
                                 uint64_t total_points, const uint64_t *sizes, int32_t n_sizes,
                                 uint64_t *out_n)
{
    if (!ctx || !plan || !kin || !pilot || !shifts || !sizes || !out_n || n_sizes < 1)
        return set_err(ctx, QMC_EINVAL, "qmc_size_lattices: null argument or no sizes");
    for (int i = 0; i < n_sizes; ++i)
        if (sizes[i] < 2 || sizes[i] >= (1ull << 31))
            return set_err(ctx, QMC_EINVAL, "qmc_size_lattices: size %llu outside [2, 2^31)",
                           (unsigned long long)sizes[i]);
    const int ns = (int)plan->secs.size();
    const int K = plan->sec_hi - plan->sec_lo + 1;
    const int no = plan->eps_hi - plan->eps_lo + 1;
    std::vector<qmc_coeff> coeff(no);
    std::vector<double> ss((size_t)ns * m * K * 2);
    qmc_result res{};
    res.coeff = coeff.data();
    res.sector_sums = ss.data();
    int rc = qmc_integrate(ctx, plan, kin, 1, pilot, nullptr, shifts, m, &res);
    if (rc) return rc;
    // kernel class of every sector at this point: deformed sectors cost more
    std::vector<double> coef(plan->n_terms), dcoef(plan->dexp.size()), w(ns);
    qmc_contract(plan, kin, coef.data(), dcoef.data());
    const double inv_n = 1.0 / (double)pilot->n;
    double wsum = 0.0;
    for (int s = 0; s < ns; ++s) {
        double spread = 0.0;
        for (int q = 0; q < K; ++q)
            for (int c = 0; c < 2; ++c) {
                double mean = 0.0;
                for (int k = 0; k < m; ++k) mean += ss[(((size_t)s * m + k) * K + q) * 2 + c];
                mean /= m;
                for (int k = 0; k < m; ++k)
                    spread = std::max(spread, std::fabs(ss[(((size_t)s * m + k) * K + q) * 2 + c] -
                                                        mean) * inv_n);
            }
        double lam = 0.0;
        const int dm = qmc_sector_mode(plan, s, coef.data(), &lam);
        const double cost = dm ? plan->secs[s].flops_deform : plan->secs[s].flops;
        spread = std::max(spread, 1e-300);
        w[s] = std::cbrt(spread * spread / cost);
        wsum += w[s];
    }
    for (int s = 0; s < ns; ++s) {
        const double want = std::max(w[s] / wsum * (double)total_points, 1.0);
        int best = 0;
        for (int i = 1; i < n_sizes; ++i)
            if (std::fabs(std::log((double)sizes[i]) - std::log(want)) <
                std::fabs(std::log((double)sizes[best]) - std::log(want)))
                best = i;
        out_n[s] = sizes[best];
    }
    return QMC_OK;
}

extern "C" int qmc_job_set_graph(qmc_job *job, int enable)
{
    if (!job) return QMC_EINVAL;
    if (job->launched) return set_err(job->ctx, QMC_EINVAL, "job is running");
    job->use_graph = enable != 0;
    if (!job->use_graph && job->graph) {
        (void)hipGraphExecDestroy(job->graph);
        job->graph = nullptr;
    }
    return QMC_OK;
}

extern "C" int qmc_job_set_variant(qmc_job *job, int32_t variant)
{
    if (!job) return QMC_EINVAL;
    if (variant != 0 && variant != 1)
        return set_err(job->ctx, QMC_EINVAL, "occupancy variant %d is not 0 or 1", variant);
    if (job->launched) return set_err(job->ctx, QMC_EINVAL, "job is running");
    for (qmc_class &c : job->classes) c.variant = variant;
    if (job->graph) {
        (void)hipGraphExecDestroy(job->graph);
        job->graph = nullptr;
    }
    return QMC_OK;
}

extern "C" int qmc_job_set_profiling(qmc_job *job, int enable)
{
    if (!job) return QMC_EINVAL;
    if (job->launched) return set_err(job->ctx, QMC_EINVAL, "job is running");
    (void)hipSetDevice(job->ctx->device);
    for (hipEvent_t e : job->ev_cls) (void)hipEventDestroy(e);
    job->ev_cls.clear();
    job->cls_timed = false;
    if (enable) {
        job->ev_cls.resize(job->classes.size() + 1, nullptr);
        for (auto &e : job->ev_cls)
            if (hipEventCreate(&e) != hipSuccess) {
                for (hipEvent_t x : job->ev_cls)
                    if (x) (void)hipEventDestroy(x);
                job->ev_cls.clear();
                return set_err(job->ctx, QMC_EDEVICE, "event creation failed");
            }
    }
    return QMC_OK;
}

extern "C" int qmc_job_class_stats(const qmc_job *job, qmc_class_stat *out, int32_t max,
                                   int32_t *n)
{
    if (!job || !n) return QMC_EINVAL;
    const int nc = (int)job->classes.size();
    for (int i = 0; i < nc && out && i < max; ++i) {
        const qmc_class &c = job->classes[i];
        const int items = c.end - c.begin;
        qmc_class_stat &st = out[i];
        st.poles = c.ks;
        st.width = c.dm;
        st.points_per_lane = c.ppl;
        st.grid = qmc_class_grid(c);
        st.items = items;
        st.precision = job->plan->opts.precision;
        st.evals = c.evals;
        st.algo_flops = c.flops;
        st.ms = (size_t)i < job->cls_ms.size() ? job->cls_ms[i] : -1.0;
        st.variant = c.variant;
        st.pad = 0;
    }
    *n = nc;
    return QMC_OK;
}

extern "C" int qmc_math_eval(qmc_ctx *ctx, int32_t fn, const double *x, double *y,
                             int64_t n)
{
    if (!ctx) return QMC_EINVAL;
    if (n < 0 || fn < QMC_MATH_LN || fn > QMC_MATH_EXPM1_F32 || (n > 0 && (!x || !y)))
        return set_err(ctx, QMC_EINVAL, "qmc_math_eval: bad argument");
    (void)hipSetDevice(ctx->device);
    HIP_CHECK(ctx, qmc_launch_math(fn, x, y, (long)n, ctx->stream));
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    return QMC_OK;
}

// Candidate launch shapes, timed per kernel class on the caller's inputs.
extern "C" int qmc_autotune(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                            int32_t n_points, const qmc_lattice *lat,
                            const qmc_lattice *lat_per_sector, const double *shifts, int32_t m,
                            qmc_tune_choice *choices, int32_t max_choices, int32_t *n_choices)
{
    if (!ctx || !plan) return QMC_EINVAL;
    // candidates in order of preference; a later one replaces the best so
    // far only when it is more than 2% faster, so that shapes whose times
    // differ by noise do not flip from one tuning to the next
    static const int ppls[] = {64, 16, 256, 4, 1024};
    static const int grids[] = {0, 4, 8};
    static const int variants[] = {0, 1};
    constexpr float margin = 0.98f;
    std::map<std::string, std::pair<qmc_tune, std::pair<int, int>>> best;
    for (int ppl : ppls) {
        qmc_job *job = nullptr;
        int rc = qmc_bind_impl(ctx, plan, kin, n_points, lat, lat_per_sector, shifts, m, ppl, 0,
                               true, &job);
        if (rc) return rc;
        uint64_t nmax = 0;
        for (uint64_t v : job->n_per_sector) nmax = std::max(nmax, v);
        bool warmed = false;
        for (int var : variants)
        for (int gpc : grids) {
            for (qmc_class &c : job->classes) {
                c.grid = gpc * ctx->n_cu;
                c.variant = var;
            }
            for (int rep = warmed ? 0 : -1; rep < 1; ++rep) {
                rc = qmc_run(job);
                if (!rc) {
                    const hipError_t e = hipStreamSynchronize(ctx->stream);
                    if (e != hipSuccess) rc = set_err(ctx, QMC_EDEVICE, "autotune: %s",
                                                      hipGetErrorString(e));
                }
                job->launched = false;
                if (rc) break;
            }
            warmed = true;
            if (rc) break;
            for (size_t i = 0; i < job->classes.size(); ++i) {
                const qmc_class &c = job->classes[i];
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, job->ev_cls[i], job->ev_cls[i + 1]) != hipSuccess)
                    continue;
                const std::string key = qmc_tune_key(plan, c.ks, c.dm, c.num, nmax);
                auto it = best.find(key);
                if (it == best.end() || ms < margin * it->second.first.ms) {
                    qmc_tune t;
                    t.ppl = ppl;
                    t.grid_per_cu = gpc;
                    t.variant = var;
                    t.ms = ms;
                    best[key] = {t, {c.ks, c.dm}};
                }
            }
        }
        qmc_job_free(job);
        if (rc) return rc;
    }
    int k = 0;
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        for (auto &kv : best) {
            ctx->tuned[kv.first] = kv.second.first;
            if (choices && k < max_choices) {
                qmc_tune_choice &ch = choices[k];
                ch.poles = kv.second.second.first;
                ch.width = kv.second.second.second;
                ch.points_per_lane = kv.second.first.ppl;
                ch.grid_per_cu = kv.second.first.grid_per_cu;
                ch.occupancy_variant = kv.second.first.variant;
                ch.pad = 0;
                ch.ms = kv.second.first.ms;
            }
            ++k;
        }
    }
    if (n_choices) *n_choices = k;
    return QMC_OK;
}
