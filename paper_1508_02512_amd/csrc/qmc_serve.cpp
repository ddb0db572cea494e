// Serving: continuous batching of integration requests.
//
// A scheduler thread per context admits queued requests (up to max_slots,
// within the HBM budget) and repeatedly launches one batch that advances
// every active request by one lattice size of its embedded rank-1 lattice
// (Section III, Eq. 17): n0 first, then n -> 2n over the odd indices only,
// since the points {2j z / 2n} of the even indices are the previous
// lattice.  Requests of different plans, kinematic points and lattice sizes
// share the launches of one batch (one launch per plan and kernel class).
// Per-shift sums stay with the request; after every batch each request is
// assembled (Eqs. 19-20) and retired once its error target is met.
//
// A request's work items, tile sizes and summation order depend only on the
// request itself, so its result is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qmc_internal.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const qmc_plan *plan = nullptr;
    std::vector<double> kin;
    double target = 1e-3;
    uint64_t n0 = 0, n_max = 0, n_cur = 0;
    int m = 0;
    uint32_t z[QMC_DMAX] = {};
    std::vector<double> shifts;          // [m][QMC_DMAX]
    std::vector<double> coef, dcoef;     // contracted at the request's point
    std::vector<double> lam;             // [ns]
    std::vector<int> dm;                 // [ns] complex kernel width or 0
    std::vector<double> hi, lo;          // running sums [ns][m][kstride][2]
    std::vector<qmc_coeff> coeff;        // current result
    uint64_t evals = 0;
    long violations = 0;
    int steps = 0;
    int halvings_left = 0, halvings = 0; // deformation back-offs (allowed, taken)
    int status = QMC_PENDING;
    bool cancelled = false, done = false;
    clk::time_point t_submit, t_done;
    // this step
    uint64_t step_n = 0, step_start = 0, step_stride = 1, step_count = 0, step_tile = 0;
    int group_base = 0;
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

} // namespace

struct qmc_serve_state {
    qmc_ctx *ctx = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool stop = false, started = false;
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    hipStream_t stream = nullptr;
    std::map<std::string, DevBuf> bufs;
    size_t pool_bytes = 0;
};

namespace {

int grow(qmc_serve_state *S, const char *name, size_t bytes, void **out)
{
    DevBuf &b = S->bufs[name];
    if (b.bytes < bytes) {
        if (b.p) {
            qmc_dev_free(S->ctx, b.p, b.bytes);
            S->pool_bytes -= b.bytes;
            b.p = nullptr;
            b.bytes = 0;
        }
        const size_t want = std::max(bytes, (size_t)4096) * 5 / 4;
        int rc = qmc_dev_alloc(S->ctx, &b.p, want);
        if (rc) return rc;
        b.bytes = want;
        S->pool_bytes += want;
    }
    *out = b.p;
    return QMC_OK;
}

void splitmix_shifts(uint64_t seed, int m, std::vector<double> &out)
{
    out.assign((size_t)m * QMC_DMAX, 0.0);
    uint64_t state = seed;
    for (size_t i = 0; i < out.size(); ++i) {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        out[i] = (double)(z >> 11) * 0x1.0p-53;
    }
}

// items (32 B) + partial slots + group sums of one step, plus rows
size_t step_bytes(const Request *r, int kstride)
{
    const size_t ns = r->plan->secs.size();
    const size_t groups = ns * r->m;
    const size_t items = groups * 6;
    return items * (sizeof(qmc_item) + (size_t)kstride * 32 + 4) +
           groups * ((size_t)kstride * 16 + 12) +
           (r->coef.size() + r->dcoef.size() + r->shifts.size() + ns) * 8 +
           ns * sizeof(qmc_lat_dev) + (size_t)(r->plan->kstride) * ns * r->m * 32;
}

void finish(qmc_serve_state *S, Request *r, int status)
{
    r->status = status;
    r->done = true;
    r->t_done = clk::now();
    (void)S;
}

bool converged(const Request *r)
{
    if (r->n_cur == 0) return false;         // restarted: no result yet
    double maxs = 0.0;
    for (const qmc_coeff &c : r->coeff) maxs = std::max(maxs, std::hypot(c.re, c.im));
    for (const qmc_coeff &c : r->coeff) {
        const double err = std::hypot(c.err_re, c.err_im);
        const double sc = std::hypot(c.re, c.im);
        const double rel = sc > 1e-3 * maxs ? err / sc : err / std::max(maxs, 1e-300);
        if (!(rel <= r->target)) return false;
    }
    return true;
}

// One batch over all active requests; returns a status for the whole batch.
int run_step(qmc_serve_state *S, std::vector<Request *> &act)
{
    qmc_ctx *ctx = S->ctx;
    // lattice stage of every request
    int kstride = 1;
    for (Request *r : act) {
        kstride = std::max(kstride, r->plan->kstride);
        if (r->n_cur == 0) {
            r->step_n = r->n0;
            r->step_start = 0;
            r->step_stride = 1;
            r->step_count = r->n0;
        } else {
            r->step_n = 2 * r->n_cur;
            r->step_start = 1;
            r->step_stride = 2;
            r->step_count = r->n_cur;
        }
        const uint64_t ppl = std::min<uint64_t>(
            std::max<uint64_t>((r->step_count + QMC_BLOCK * 4 - 1) / (QMC_BLOCK * 4), 1), 1 << 14);
        r->step_tile = (uint64_t)QMC_BLOCK * ppl;
    }
    // requests by plan; rows of the per-plan input blocks
    std::vector<const qmc_plan *> plans;
    for (Request *r : act)
        if (std::find(plans.begin(), plans.end(), r->plan) == plans.end()) plans.push_back(r->plan);
    struct PlanBlock {
        std::vector<Request *> reqs;
        size_t coef_off = 0, dcoef_off = 0, shift_off = 0, lam_off = 0, lat_off = 0;
    };
    std::vector<PlanBlock> blocks(plans.size());
    std::vector<double> coef, dcoef, shifts, lam;
    std::vector<qmc_lat_dev> lats;
    int groups = 0;
    for (size_t pi = 0; pi < plans.size(); ++pi) {
        PlanBlock &B = blocks[pi];
        for (Request *r : act)
            if (r->plan == plans[pi]) B.reqs.push_back(r);
        B.coef_off = coef.size();
        B.dcoef_off = dcoef.size();
        B.shift_off = shifts.size();
        B.lam_off = lam.size();
        B.lat_off = lats.size();
        for (Request *r : B.reqs) {
            coef.insert(coef.end(), r->coef.begin(), r->coef.end());
            dcoef.insert(dcoef.end(), r->dcoef.begin(), r->dcoef.end());
            shifts.insert(shifts.end(), r->shifts.begin(), r->shifts.end());
            lam.insert(lam.end(), r->lam.begin(), r->lam.end());
            const int ns = (int)r->plan->secs.size();
            for (int s = 0; s < ns; ++s) {
                const qmc_sec_host &h = r->plan->secs[s];
                qmc_lat_dev d{};
                d.n = (uint32_t)r->step_n;
                d.inv_n = 1.0 / (double)r->step_n;
                for (int j = 0; j < QMC_DMAX; ++j)
                    d.z[j] = j < h.dim ? (uint32_t)(r->z[h.perm[j]] % r->step_n) : 0u;
                lats.push_back(d);
            }
            r->group_base = groups;
            groups += ns * r->m;
        }
    }
    // items grouped by (plan, kernel class)
    std::vector<qmc_item> items;
    std::vector<int32_t> gbeg(groups), gend(groups);
    struct Launch {
        size_t plan;
        qmc_class cls;
    };
    std::vector<Launch> launches;
    for (size_t pi = 0; pi < plans.size(); ++pi) {
        const qmc_plan *P = plans[pi];
        const int ns = (int)P->secs.size();
        std::vector<std::pair<int, int>> keys;
        for (Request *r : blocks[pi].reqs)
            for (int s = 0; s < ns; ++s) {
                std::pair<int, int> key{P->secs[s].ks, r->dm[s]};
                if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
            }
        std::sort(keys.begin(), keys.end());
        for (const auto &key : keys) {
            qmc_class c{};
            c.ks = key.first;
            c.dm = key.second;
            c.deform = c.dm != 0;
            c.kb = P->kb;
            c.begin = (int)items.size();
            for (size_t row = 0; row < blocks[pi].reqs.size(); ++row) {
                Request *r = blocks[pi].reqs[row];
                for (int s = 0; s < ns; ++s) {
                    if (P->secs[s].ks != c.ks || r->dm[s] != c.dm) continue;
                    for (int k = 0; k < r->m; ++k) {
                        const int g = r->group_base + s * r->m + k;
                        gbeg[g] = (int32_t)items.size();
                        for (uint64_t off = 0; off < r->step_count; off += r->step_tile) {
                            qmc_item it{};
                            it.sector = s;
                            it.point = (int32_t)row;
                            it.shift = (int32_t)(row * r->m + k);
                            it.group = g;
                            it.lat = (int32_t)(row * ns + s);
                            it.start = (uint32_t)(r->step_start + r->step_stride * off);
                            it.count = (uint32_t)std::min<uint64_t>(r->step_tile,
                                                                    r->step_count - off);
                            it.stride = (uint32_t)r->step_stride;
                            items.push_back(it);
                        }
                        gend[g] = (int32_t)items.size();
                    }
                }
            }
            c.end = (int)items.size();
            if (c.end > c.begin) launches.push_back({pi, c});
        }
    }
    // device buffers (grow-only pools) and uploads
    void *d_items, *d_gbeg, *d_gend, *d_partial, *d_viol, *d_out, *d_gviol;
    void *d_coef, *d_dcoef, *d_shift, *d_lam, *d_lat;
    int rc = QMC_OK;
    rc = rc ? rc : grow(S, "items", items.size() * sizeof(qmc_item), &d_items);
    rc = rc ? rc : grow(S, "gbeg", groups * 4, &d_gbeg);
    rc = rc ? rc : grow(S, "gend", groups * 4, &d_gend);
    rc = rc ? rc : grow(S, "partial", items.size() * (size_t)kstride * 32, &d_partial);
    rc = rc ? rc : grow(S, "viol", items.size() * 4, &d_viol);
    rc = rc ? rc : grow(S, "out", (size_t)groups * kstride * 16, &d_out);
    rc = rc ? rc : grow(S, "gviol", groups * 4, &d_gviol);
    rc = rc ? rc : grow(S, "coef", coef.size() * 8, &d_coef);
    rc = rc ? rc : grow(S, "dcoef", dcoef.size() * 8, &d_dcoef);
    rc = rc ? rc : grow(S, "shift", shifts.size() * 8, &d_shift);
    rc = rc ? rc : grow(S, "lam", lam.size() * 8, &d_lam);
    rc = rc ? rc : grow(S, "lat", lats.size() * sizeof(qmc_lat_dev), &d_lat);
    if (rc) return rc;
    hipStream_t st = S->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t e = up(d_items, items.data(), items.size() * sizeof(qmc_item));
    if (e == hipSuccess) e = up(d_gbeg, gbeg.data(), groups * 4);
    if (e == hipSuccess) e = up(d_gend, gend.data(), groups * 4);
    if (e == hipSuccess) e = up(d_coef, coef.data(), coef.size() * 8);
    if (e == hipSuccess) e = up(d_dcoef, dcoef.data(), dcoef.size() * 8);
    if (e == hipSuccess) e = up(d_shift, shifts.data(), shifts.size() * 8);
    if (e == hipSuccess) e = up(d_lam, lam.data(), lam.size() * 8);
    if (e == hipSuccess) e = up(d_lat, lats.data(), lats.size() * sizeof(qmc_lat_dev));
    for (const Launch &L : launches) {
        if (e != hipSuccess) break;
        const qmc_plan *P = plans[L.plan];
        const PlanBlock &B = blocks[L.plan];
        qmc_launch_args A{};
        A.sec = P->d_sec;
        A.lat = (const qmc_lat_dev *)d_lat + B.lat_off;
        A.texp = P->d_texp;
        A.texpd = P->d_texpd;
        A.tprog = P->d_tprog;
        A.dprog = P->d_dprog;
        A.tcoef = (const double *)d_coef + B.coef_off;
        A.dexp = P->d_dexp;
        A.dcoef = (const double *)d_dcoef + B.dcoef_off;
        A.shifts = (const double *)d_shift + B.shift_off;
        A.lam = (const double *)d_lam + B.lam_off;
        A.items = (const qmc_item *)d_items;
        A.partial = (double *)d_partial;
        A.viol = (int32_t *)d_viol;
        A.n_terms = P->n_terms;
        A.n_dterms = (int32_t)P->dexp.size();
        A.item_begin = L.cls.begin;
        A.item_end = L.cls.end;
        A.kstride = kstride;
        A.korobov_r = P->opts.korobov_r;
        A.n_sec = (int32_t)P->secs.size();
        e = qmc_launch_class(P, L.cls, A, st);
    }
    if (e == hipSuccess)
        e = qmc_launch_reduce((const double *)d_partial, (const int32_t *)d_viol,
                              (const int32_t *)d_gbeg, (const int32_t *)d_gend, groups, kstride,
                              (double *)d_out, (int32_t *)d_gviol, st);
    std::vector<double> out((size_t)groups * kstride * 2);
    std::vector<int32_t> gviol(groups);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out.data(), d_out, out.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(gviol.data(), d_gviol, groups * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return qmc_set_error(ctx, QMC_EDEVICE, "serving step: %s", hipGetErrorString(e));
    // fold the batch into every request and assemble
    for (Request *r : act) {
        const qmc_plan *P = r->plan;
        const int ns = (int)P->secs.size();
        r->evals += r->step_count * (uint64_t)ns * r->m;
        r->steps += 1;
        // sign violations of the deformed contour: back off lambda in the
        // sectors concerned and restart the request while back-offs remain
        std::vector<long> vsec(ns, 0);
        long vtot = 0;
        for (int s = 0; s < ns; ++s)
            for (int k = 0; k < r->m; ++k) {
                vsec[s] += gviol[r->group_base + s * r->m + k];
                vtot += gviol[r->group_base + s * r->m + k];
            }
        if (vtot > 0 && r->halvings_left > 0) {
            for (int s = 0; s < ns; ++s)
                if (vsec[s] > 0) r->lam[s] *= 0.5;
            r->halvings_left -= 1;
            r->halvings += 1;
            std::fill(r->hi.begin(), r->hi.end(), 0.0);
            std::fill(r->lo.begin(), r->lo.end(), 0.0);
            r->n_cur = 0;                    // the next step starts again at n0
            continue;
        }
        r->violations += vtot;
        for (int s = 0; s < ns; ++s)
            for (int k = 0; k < r->m; ++k) {
                const int g = r->group_base + s * r->m + k;
                for (int q = 0; q < P->kstride * 2; ++q) {
                    const size_t o = ((size_t)(s * r->m + k) * P->kstride * 2) + q;
                    const double x = out[(size_t)g * kstride * 2 + q];
                    const double a = r->hi[o], sum = a + x, bb = sum - a;
                    r->lo[o] += (a - (sum - bb)) + (x - bb);
                    r->hi[o] = sum;
                }
            }
        r->n_cur = r->step_n;
        std::vector<double> gsum(r->hi.size());
        for (size_t i = 0; i < gsum.size(); ++i) gsum[i] = r->hi[i] + r->lo[i];
        std::vector<uint64_t> nsec(ns, r->n_cur);
        qmc_result res{};
        res.coeff = r->coeff.data();
        qmc_assemble(P, 1, r->m, nsec, gsum.data(), &res);
    }
    return QMC_OK;
}

void scheduler(qmc_serve_state *S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->active.empty(); });
        if (S->stop) break;
        // cancellations
        for (auto it = S->active.begin(); it != S->active.end();) {
            if ((*it)->cancelled) {
                finish(S, *it, QMC_ECANCELLED);
                it = S->active.erase(it);
            } else {
                ++it;
            }
        }
        while (!S->pending.empty() && S->pending.front()->cancelled) {
            finish(S, S->pending.front(), QMC_ECANCELLED);
            S->pending.pop_front();
        }
        // admission by slots and device memory
        size_t need = 0;
        for (Request *r : S->active) need += step_bytes(r, QMC_MAX_ORDERS);
        while (!S->pending.empty() && (int)S->active.size() < S->ctx->max_slots) {
            Request *r = S->pending.front();
            const size_t more = step_bytes(r, QMC_MAX_ORDERS);
            const size_t other = S->ctx->used.load() - S->pool_bytes;
            const size_t avail = S->ctx->budget > other ? S->ctx->budget - other : 0;
            if (need + more > avail) {
                if (S->active.empty()) {         // cannot fit even alone
                    qmc_set_error(S->ctx, QMC_EBUDGET, "request %llu does not fit the budget",
                                  (unsigned long long)r->ticket);
                    finish(S, r, QMC_EBUDGET);
                    S->pending.pop_front();
                    continue;
                }
                break;
            }
            need += more;
            S->active.push_back(r);
            S->pending.pop_front();
        }
        S->done_cv.notify_all();
        if (S->active.empty()) continue;
        std::vector<Request *> act = S->active;
        lk.unlock();
        const int rc = run_step(S, act);
        lk.lock();
        for (auto it = S->active.begin(); it != S->active.end();) {
            Request *r = *it;
            bool retire = false;
            if (rc != QMC_OK) {
                finish(S, r, rc);
                retire = true;
            } else if (r->violations > 0) {
                finish(S, r, QMC_EDEFORM);
                retire = true;
            } else if (converged(r)) {
                finish(S, r, QMC_OK);
                retire = true;
            } else if (2 * r->n_cur > r->n_max) {
                finish(S, r, QMC_ENOTCONVERGED);
                retire = true;
            }
            it = retire ? S->active.erase(it) : it + 1;
        }
        S->done_cv.notify_all();
    }
    // drain
    for (Request *r : S->active) finish(S, r, QMC_ECANCELLED);
    for (Request *r : S->pending) finish(S, r, QMC_ECANCELLED);
    S->active.clear();
    S->pending.clear();
    S->done_cv.notify_all();
}

qmc_serve_state *serve_state(qmc_ctx *ctx)
{
    std::lock_guard<std::mutex> g(ctx->serve_mu);
    if (!ctx->serve) {
        auto *S = new qmc_serve_state();
        S->ctx = ctx;
        (void)hipSetDevice(ctx->device);
        if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
            delete S;
            return nullptr;
        }
        S->th = std::thread(scheduler, S);
        S->started = true;
        ctx->serve = S;
    }
    return ctx->serve;
}

void fill(const Request *r, qmc_result *out)
{
    if (!out) return;
    if (out->coeff)
        std::copy(r->coeff.begin(), r->coeff.end(), out->coeff);
    out->evals = r->evals;
    out->n_final = r->n_cur;
    out->status = r->status;
    out->deform_violations = (int32_t)std::min<long>(r->violations, INT32_MAX);
    out->kernel_ms = 0.0;
    out->algo_flops = 0.0;
    out->latency_ms =
        std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    out->steps = r->steps;
    out->lambda_halvings = r->halvings;
}

} // namespace

void qmc_serve_shutdown(qmc_ctx *ctx)
{
    qmc_serve_state *S = ctx->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    for (auto &kv : S->all) delete kv.second;
    for (auto &kv : S->bufs) qmc_dev_free(ctx, kv.second.p, kv.second.bytes);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    ctx->serve = nullptr;
}

extern "C" int qmc_submit(qmc_ctx *ctx, const qmc_plan *plan, const qmc_request *req,
                          uint64_t *ticket)
{
    if (!ctx || !plan || !req || !ticket || !req->kin || !req->z)
        return qmc_set_error(ctx, QMC_EINVAL, "null argument");
    if (req->m < 2) return qmc_set_error(ctx, QMC_EINVAL, "need m >= 2 shifts");
    auto pow2 = [](uint64_t v) { return v >= 2 && (v & (v - 1)) == 0; };
    if (!pow2(req->n0) || !pow2(req->n_max) || req->n0 > req->n_max ||
        req->n_max >= (1ull << 31))
        return qmc_set_error(ctx, QMC_EINVAL, "n0 <= n_max must be powers of two below 2^31");
    if (!(req->rel_err_target > 0.0))
        return qmc_set_error(ctx, QMC_EINVAL, "rel_err_target must be positive");
    if (req->lambda_halvings < 0 || req->lambda_halvings > 16)
        return qmc_set_error(ctx, QMC_EINVAL, "lambda_halvings must be in 0..16");
    for (int j = 0; j < QMC_DMAX; ++j)
        if ((req->z[j] & 1u) == 0u)
            return qmc_set_error(ctx, QMC_EINVAL, "z must be odd (coprime to 2^k)");
    qmc_serve_state *S = serve_state(ctx);
    if (!S) return qmc_set_error(ctx, QMC_EDEVICE, "cannot start the scheduler");
    auto *r = new (std::nothrow) Request();
    if (!r) return qmc_set_error(ctx, QMC_ENOMEM, "host allocation");
    r->plan = plan;
    r->kin.assign(req->kin, req->kin + plan->n_inv);
    r->target = req->rel_err_target;
    r->n0 = req->n0;
    r->n_max = req->n_max;
    r->m = req->m;
    r->halvings_left = req->lambda_halvings;
    std::memcpy(r->z, req->z, sizeof r->z);
    splitmix_shifts(req->seed, r->m, r->shifts);
    const int ns = (int)plan->secs.size();
    r->coef.resize(plan->n_terms);
    r->dcoef.resize(plan->dexp.size());
    qmc_contract(plan, r->kin.data(), r->coef.data(), r->dcoef.data());
    r->lam.resize(ns);
    r->dm.resize(ns);
    for (int s = 0; s < ns; ++s) r->dm[s] = qmc_sector_mode(plan, s, r->coef.data(), &r->lam[s]);
    r->hi.assign((size_t)ns * r->m * plan->kstride * 2, 0.0);
    r->lo.assign(r->hi.size(), 0.0);
    r->coeff.assign(plan->eps_hi - plan->eps_lo + 1, qmc_coeff{});
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> g(S->mu);
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        S->pending.push_back(r);
    }
    S->cv.notify_all();
    *ticket = r->ticket;
    return QMC_OK;
}

extern "C" int qmc_poll(qmc_ctx *ctx, uint64_t ticket, qmc_result *out)
{
    if (!ctx || !ctx->serve) return QMC_EINVAL;
    qmc_serve_state *S = ctx->serve;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return QMC_EINVAL;
    if (!it->second->done) return QMC_PENDING;
    fill(it->second, out);
    return it->second->status;
}

extern "C" int qmc_wait(qmc_ctx *ctx, uint64_t ticket, double timeout_s, qmc_result *out)
{
    if (!ctx || !ctx->serve) return QMC_EINVAL;
    qmc_serve_state *S = ctx->serve;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return QMC_EINVAL;
    Request *r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_s < 0) {
        S->done_cv.wait(lk, ready);
    } else if (!S->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return QMC_PENDING;
    }
    fill(r, out);
    return r->status;
}

extern "C" int qmc_cancel(qmc_ctx *ctx, uint64_t ticket)
{
    if (!ctx || !ctx->serve) return QMC_EINVAL;
    qmc_serve_state *S = ctx->serve;
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return QMC_EINVAL;
        it->second->cancelled = true;
    }
    S->cv.notify_all();
    return QMC_OK;
}

extern "C" int qmc_release(qmc_ctx *ctx, uint64_t ticket)
{
    if (!ctx || !ctx->serve) return QMC_EINVAL;
    qmc_serve_state *S = ctx->serve;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return QMC_EINVAL;
    if (!it->second->done) return QMC_PENDING;
    delete it->second;
    S->all.erase(it);
    return QMC_OK;
}
