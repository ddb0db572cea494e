// Serving: continuous batching of integration requests.
//
// A scheduler thread per context admits queued requests (up to max_slots,
// within the HBM budget) and runs batch steps.  Each request integrates an
// embedded rank-1 lattice (Section III, Eq. 17) level by level: n0 first,
// then n -> 2n over the odd indices only, since the points {2j z / 2n} of
// the even indices are the previous level.  A step advances every active
// request by an equal share of a fixed work budget (2^26 evaluations), so
// a step, and the wait of a new arrival for admission, stays bounded; a
// level may take several steps.
//
// Per-request state is resident on the device from admission to
// retirement: the contracted coefficients, lambda per sector, the shifts
// and the level's lattice rows (rows of slot-indexed pools), and the
// compensated per-(sector, shift, order) sums, to which every step adds its
// work items one by one in item order.  When a level completes, a small kernel
// combines the sectors per shift and only m x orders values come back for
// the mean and error (Eqs. 19-20) and the convergence check.
//
// A request's work items and their summation order depend only on the
// request itself (not on how its levels are cut into steps, which depends
// on the load), so its result is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
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

// Work of one batch step: at most this many integrand evaluations (whole
// work items), shared evenly by the active requests, so that a step, and
// hence the wait of a newly arrived request for admission, stays bounded
// whatever the lattice sizes of the requests already running.  Work items
// are tiles of SERVE_TILE lattice indices (32 per lane), small enough that a
// step has thousands of work-groups.
constexpr uint64_t STEP_EVALS = 1ull << 26;
constexpr uint64_t SERVE_TILE = (uint64_t)QMC_BLOCK * 32;
constexpr int MAX_SHIFTS = 64;           // shift rows per request slot

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Device rows of one plan, one per request slot: contracted coefficients,
// derivative coefficients, per-sector lambda and per-sector lattices of the
// request's current level; plus the sector constants D.
struct PlanPool {
    const qmc_plan *plan = nullptr;
    DevBuf coef, dcoef, lam, lat, D;
    int refs = 0;                        // active requests of the plan
};

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
    std::vector<qmc_coeff> coeff;        // current result
    uint64_t evals = 0;
    long violations = 0;
    int steps = 0;
    int halvings_left = 0, halvings = 0; // deformation back-offs (allowed, taken)
    int status = QMC_PENDING;
    bool cancelled = false, done = false;
    clk::time_point t_submit, t_done;
    // resident device state
    int slot = -1;                       // row in the plan pool and shift pool
    DevBuf sums;                         // [ns][m][kstride][4] compensated sums
    size_t mem = 0;                      // bytes admitted for this request
    // current level: n = level_n, indices start, start + stride, ...
    uint64_t level_n = 0, level_start = 0, level_stride = 1, level_count = 0, tile = 0;
    uint64_t items_per_group = 0, level_items = 0, cursor = 0;
    bool level_fresh = true;             // lattice rows of this level not uploaded yet
    long level_viol = 0;
    std::vector<long> level_vsec;        // violations per sector in this level
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
    std::map<std::string, DevBuf> bufs;  // step buffers (grow-only)
    std::map<const qmc_plan *, PlanPool> pools;
    DevBuf shift_pool;                   // [max_slots][MAX_SHIFTS][QMC_DMAX]
    std::vector<int> free_slots;
    size_t pool_bytes = 0;               // device bytes of everything above
    size_t fixed_bytes = 0;              // of which plan pools and the shift pool
    size_t admitted = 0;                 // bytes admitted for active requests
};

namespace {

int dev_alloc(qmc_serve_state *S, DevBuf &b, size_t bytes)
{
    b.p = nullptr;
    b.bytes = 0;
    if (bytes == 0) return QMC_OK;
    int rc = qmc_dev_alloc(S->ctx, &b.p, bytes);
    if (rc) return rc;
    b.bytes = bytes;
    S->pool_bytes += bytes;
    return QMC_OK;
}

void dev_free(qmc_serve_state *S, DevBuf &b)
{
    if (!b.p) return;
    qmc_dev_free(S->ctx, b.p, b.bytes);
    S->pool_bytes -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

int grow(qmc_serve_state *S, const char *name, size_t bytes, void **out)
{
    DevBuf &b = S->bufs[name];
    if (b.bytes < bytes) {
        dev_free(S, b);
        int rc = dev_alloc(S, b, std::max(bytes, (size_t)4096) * 5 / 4);
        if (rc) return rc;
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

// Lattice indices of the level at size n: all n of them for the first
// level, else the n/2 odd ones (the even ones are the previous level).
void level_shape(uint64_t n, bool first, uint64_t &start, uint64_t &stride, uint64_t &count,
                 uint64_t &tile)
{
    start = first ? 0 : 1;
    stride = first ? 1 : 2;
    count = first ? n : n / 2;
    tile = SERVE_TILE;
}

// Items one request may take in a step when `active` requests share it
uint64_t step_items(uint64_t tile, size_t active)
{
    return std::max<uint64_t>(STEP_EVALS / (tile * std::max<size_t>(active, 1)), 1);
}

// Device bytes a request holds while active: its resident sums plus its
// largest share of the step buffers (items, partial slots, counters, group
// ranges and destinations).  A step holds min(quota, items of the level) of
// the request's items, maximised here over its levels n0 .. n_max.  Partial
// slots are sized for the widest plan a step may mix (QMC_MAX_ORDERS).
size_t request_bytes(const qmc_plan *P, int m, uint64_t n0, uint64_t n_max)
{
    const size_t ns = P->secs.size();
    const size_t groups = ns * (size_t)m;
    size_t items = 1;
    for (uint64_t n = n0; n <= n_max; n *= 2) {
        uint64_t st, sd, cnt, tile;
        level_shape(n, n == n0, st, sd, cnt, tile);
        const uint64_t level = (cnt + tile - 1) / tile * groups;
        items = std::max<size_t>(items, (size_t)std::min(step_items(tile, 1), level));
    }
    const size_t ks = (size_t)P->kstride;
    // step buffers grow by a quarter beyond what they hold
    const size_t step = items * (sizeof(qmc_item) + (size_t)QMC_MAX_ORDERS * 32 + 4) +
                        items * (4 + 4 + 8 + 4 + 4) +          // group ranges, destinations
                        (size_t)m * (P->tot_hi - P->tot_lo + 1) * 16;   // combined totals
    return groups * ks * 32 + step * 5 / 4 + 3 * 4096;
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

// Per-shift Laurent series (prefactor times the combined sector sums), then
// mean and error over the shifts (Eqs. 19-20).  tot: [m][orders tot_lo..tot_hi][2].
void assemble_totals(const qmc_plan *P, int m, const std::vector<double> &tot,
                     std::vector<qmc_coeff> &coeff)
{
    const int K = P->tot_hi - P->tot_lo + 1;
    const int no = P->eps_hi - P->eps_lo + 1;
    std::vector<std::complex<double>> Q((size_t)m * no);
    for (int k = 0; k < m; ++k)
        for (int oi = 0; oi < no; ++oi) {
            const int order = P->eps_lo + oi;
            std::complex<double> acc = 0.0;
            for (int j = 0; j < K; ++j) {
                const int pp = order - (P->tot_lo + j) - P->eps_pref_lo;
                if (pp < 0 || pp >= P->n_pref) continue;
                const std::complex<double> v(tot[((size_t)k * K + j) * 2],
                                             tot[((size_t)k * K + j) * 2 + 1]);
                acc += std::complex<double>(P->pref[2 * pp], P->pref[2 * pp + 1]) * v;
            }
            Q[(size_t)k * no + oi] = acc;
        }
    coeff.assign(no, qmc_coeff{});
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
        coeff[oi] = {mr, mi, std::sqrt(vr / ((double)m * (m - 1))),
                     std::sqrt(vi / ((double)m * (m - 1)))};
    }
}

// Device bytes of a plan's pool (all slots) and of the shift pool.
size_t plan_pool_bytes(const qmc_plan *P, int slots)
{
    const size_t ns = P->secs.size();
    return (size_t)slots * (std::max(P->n_terms, 1) + std::max<size_t>(P->dexp.size(), 1) + ns) * 8 +
           (size_t)slots * ns * sizeof(qmc_lat_dev) + ns * 16;
}

size_t shift_pool_bytes(int slots) { return (size_t)slots * MAX_SHIFTS * QMC_DMAX * 8; }

// Device rows for a request at admission: plan pool (created on the plan's
// first request), shift rows, resident sums.
int admit_device(qmc_serve_state *S, Request *r)
{
    const qmc_plan *P = r->plan;
    const int ns = (int)P->secs.size();
    const int slots = S->ctx->max_slots;
    hipStream_t st = S->stream;
    if (!S->shift_pool.p) {
        int rc = dev_alloc(S, S->shift_pool, shift_pool_bytes(slots));
        if (rc) return rc;
        S->fixed_bytes += S->shift_pool.bytes;
        S->free_slots.clear();
        for (int i = slots - 1; i >= 0; --i) S->free_slots.push_back(i);
    }
    auto it = S->pools.find(P);
    if (it == S->pools.end()) {
        PlanPool pp;
        pp.plan = P;
        int rc = dev_alloc(S, pp.coef, (size_t)slots * std::max(P->n_terms, 1) * 8);
        if (!rc) rc = dev_alloc(S, pp.dcoef, (size_t)slots * std::max<size_t>(P->dexp.size(), 1) * 8);
        if (!rc) rc = dev_alloc(S, pp.lam, (size_t)slots * ns * 8);
        if (!rc) rc = dev_alloc(S, pp.lat, (size_t)slots * ns * sizeof(qmc_lat_dev));
        // coefficient series C(eps) of every sector: [ns][QMC_MAX_ORDERS][2]
        if (!rc) rc = dev_alloc(S, pp.D, (size_t)ns * QMC_MAX_ORDERS * 16);
        std::vector<double> D((size_t)2 * ns * QMC_MAX_ORDERS, 0.0);
        for (int s = 0; s < ns; ++s)
            for (size_t e = 0; e < P->secs[s].C.size() && e < (size_t)QMC_MAX_ORDERS; ++e) {
                D[2 * ((size_t)s * QMC_MAX_ORDERS + e)] = P->secs[s].C[e].real();
                D[2 * ((size_t)s * QMC_MAX_ORDERS + e) + 1] = P->secs[s].C[e].imag();
            }
        if (!rc && hipMemcpyAsync(pp.D.p, D.data(), D.size() * 8, hipMemcpyHostToDevice, st) !=
                       hipSuccess)
            rc = QMC_EDEVICE;
        // D is a local: wait for its upload before it goes out of scope
        if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = QMC_EDEVICE;
        if (rc) {
            dev_free(S, pp.coef);
            dev_free(S, pp.dcoef);
            dev_free(S, pp.lam);
            dev_free(S, pp.lat);
            dev_free(S, pp.D);
            return rc;
        }
        S->fixed_bytes += pp.coef.bytes + pp.dcoef.bytes + pp.lam.bytes + pp.lat.bytes + pp.D.bytes;
        it = S->pools.emplace(P, pp).first;
    }
    if (S->free_slots.empty()) return QMC_EBUDGET;
    int rc = dev_alloc(S, r->sums, (size_t)ns * r->m * P->kstride * 32);
    if (rc) return rc;
    r->slot = S->free_slots.back();
    S->free_slots.pop_back();
    it->second.refs += 1;
    PlanPool &pp = it->second;
    auto up = [&](void *base, size_t row_bytes, const void *src) {
        return row_bytes ? hipMemcpyAsync((char *)base + (size_t)r->slot * row_bytes, src,
                                          row_bytes, hipMemcpyHostToDevice, st)
                         : hipSuccess;
    };
    hipError_t e = up(pp.coef.p, (size_t)P->n_terms * 8, r->coef.data());
    if (e == hipSuccess) e = up(pp.dcoef.p, P->dexp.size() * 8, r->dcoef.data());
    if (e == hipSuccess) e = up(pp.lam.p, (size_t)ns * 8, r->lam.data());
    if (e == hipSuccess)
        e = hipMemcpyAsync((char *)S->shift_pool.p + (size_t)r->slot * MAX_SHIFTS * QMC_DMAX * 8,
                           r->shifts.data(), r->shifts.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = qmc_launch_fill((double *)r->sums.p, (long)(r->sums.bytes / 8), 0.0, st);
    // the request's host rows stay alive while it is active, but a restart
    // rewrites lam: keep the uploads ordered before any later host change
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? QMC_OK : QMC_EDEVICE;
}

void release_device(qmc_serve_state *S, Request *r)
{
    if (r->slot < 0) return;
    dev_free(S, r->sums);
    S->free_slots.push_back(r->slot);
    r->slot = -1;
    auto it = S->pools.find(r->plan);
    if (it != S->pools.end() && --it->second.refs == 0) {
        PlanPool &pp = it->second;
        S->fixed_bytes -= pp.coef.bytes + pp.dcoef.bytes + pp.lam.bytes + pp.lat.bytes + pp.D.bytes;
        dev_free(S, pp.coef);
        dev_free(S, pp.dcoef);
        dev_free(S, pp.lam);
        dev_free(S, pp.lat);
        dev_free(S, pp.D);
        S->pools.erase(it);
    }
    S->admitted -= r->mem;
    r->mem = 0;
}

// Sets up the next level of a request (after admission, a completed level
// or a restart).
void start_level(Request *r)
{
    const bool first = r->n_cur == 0;
    r->level_n = first ? r->n0 : 2 * r->n_cur;
    level_shape(r->level_n, first, r->level_start, r->level_stride, r->level_count, r->tile);
    r->items_per_group = (r->level_count + r->tile - 1) / r->tile;
    r->level_items = r->items_per_group * r->plan->secs.size() * r->m;
    r->cursor = 0;
    r->level_fresh = true;
    r->level_viol = 0;
    r->level_vsec.assign(r->plan->secs.size(), 0);
}

// One batch step over all active requests: each advances by its own quota
// of work items of its current level.  Returns a status for the whole step.
int run_step(qmc_serve_state *S, std::vector<Request *> &act, std::vector<Request *> &done_lv)
{
    qmc_ctx *ctx = S->ctx;
    hipStream_t st = S->stream;
    int kstride = 1;
    for (Request *r : act) kstride = std::max(kstride, r->plan->kstride);
    // lattice rows of levels that start now
    for (Request *r : act) {
        if (!r->level_fresh) continue;
        const qmc_plan *P = r->plan;
        const int ns = (int)P->secs.size();
        std::vector<qmc_lat_dev> lats(ns);
        for (int s = 0; s < ns; ++s) {
            const qmc_sec_host &h = P->secs[s];
            qmc_lat_dev d{};
            d.n = (uint32_t)r->level_n;
            d.inv_n = 1.0 / (double)r->level_n;
            for (int j = 0; j < QMC_DMAX; ++j)
                d.z[j] = j < h.dim ? (uint32_t)(r->z[h.perm[j]] % r->level_n) : 0u;
            lats[s] = d;
        }
        PlanPool &pp = S->pools[P];
        const size_t row = (size_t)ns * sizeof(qmc_lat_dev);
        hipError_t e = hipMemcpyAsync((char *)pp.lat.p + (size_t)r->slot * row, lats.data(), row,
                                      hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);       // lats is a local
        if (e != hipSuccess)
            return qmc_set_error(ctx, QMC_EDEVICE, "serving: %s", hipGetErrorString(e));
        r->level_fresh = false;
    }
    // this step's window [cursor, cursor + quota) of every request's level,
    // items listed group-major; grouped into launches by (plan, class)
    struct Win {
        Request *r;
        uint64_t begin, end;
    };
    std::vector<Win> wins;
    for (Request *r : act) {
        const uint64_t q = step_items(r->tile, act.size());
        wins.push_back({r, r->cursor, std::min(r->cursor + q, r->level_items)});
    }
    std::vector<const qmc_plan *> plans;
    for (Request *r : act)
        if (std::find(plans.begin(), plans.end(), r->plan) == plans.end()) plans.push_back(r->plan);
    std::vector<qmc_item> items;
    std::vector<int32_t> gbeg, gend;
    std::vector<double *> gdst;
    std::vector<int32_t> gks;                      // order slots of each group's sums
    std::vector<std::pair<Request *, int>> gown;   // (request, sector) of each step group
    struct Launch {
        const qmc_plan *plan;
        qmc_class cls;
    };
    std::vector<Launch> launches;
    for (const qmc_plan *P : plans) {
        const int ns = (int)P->secs.size();
        // (poles, kernel width or 0, numerator factors or not)
        std::vector<std::array<int, 3>> keys;
        for (const Win &w : wins) {
            if (w.r->plan != P) continue;
            for (int s = 0; s < ns; ++s) {
                std::array<int, 3> key{P->secs[s].ks, w.r->dm[s], qmc_num_class(P, s)};
                if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
            }
        }
        std::sort(keys.begin(), keys.end());
        for (const auto &key : keys) {
            qmc_class c{};
            c.ks = key[0];
            c.dm = key[1];
            c.num = key[2];
            c.deform = c.dm != 0;
            c.kb = P->kb;
            c.begin = (int)items.size();
            for (const Win &w : wins) {
                Request *r = w.r;
                if (r->plan != P || w.end <= w.begin) continue;
                const uint64_t ipg = r->items_per_group;
                const uint64_t g0 = w.begin / ipg, g1 = (w.end - 1) / ipg;
                for (uint64_t g = g0; g <= g1; ++g) {
                    const int s = (int)(g / r->m), k = (int)(g % r->m);
                    if (P->secs[s].ks != c.ks || r->dm[s] != c.dm || qmc_num_class(P, s) != c.num)
                        continue;
                    gbeg.push_back((int32_t)items.size());
                    const uint64_t i0 = std::max(w.begin, g * ipg), i1 = std::min(w.end, (g + 1) * ipg);
                    for (uint64_t i = i0; i < i1; ++i) {
                        const uint64_t off = (i - g * ipg) * r->tile;
                        qmc_item it{};
                        it.sector = s;
                        it.point = r->slot;
                        it.shift = r->slot * MAX_SHIFTS + k;
                        it.group = (int32_t)gbeg.size() - 1;
                        it.lat = r->slot * ns + s;
                        it.start = (uint32_t)(r->level_start + r->level_stride * off);
                        it.count = (uint32_t)std::min<uint64_t>(r->tile, r->level_count - off);
                        it.stride = (uint32_t)r->level_stride;
                        items.push_back(it);
                        c.evals += it.count;
                    }
                    gend.push_back((int32_t)items.size());
                    gdst.push_back((double *)r->sums.p + ((size_t)(s * r->m + k) * P->kstride) * 4);
                    gks.push_back(P->kstride);
                    gown.push_back({r, s});
                }
            }
            c.end = (int)items.size();
            if (c.end > c.begin) launches.push_back({P, c});
        }
    }
    const int groups = (int)gbeg.size();
    void *d_items, *d_gbeg, *d_gend, *d_gdst, *d_gks, *d_partial, *d_viol, *d_gviol;
    int rc = QMC_OK;
    rc = rc ? rc : grow(S, "items", items.size() * sizeof(qmc_item), &d_items);
    rc = rc ? rc : grow(S, "gbeg", (size_t)groups * 4, &d_gbeg);
    rc = rc ? rc : grow(S, "gend", (size_t)groups * 4, &d_gend);
    rc = rc ? rc : grow(S, "gdst", (size_t)groups * 8, &d_gdst);
    rc = rc ? rc : grow(S, "gks", (size_t)groups * 4, &d_gks);
    rc = rc ? rc : grow(S, "partial", items.size() * (size_t)kstride * 32, &d_partial);
    rc = rc ? rc : grow(S, "viol", items.size() * 4, &d_viol);
    rc = rc ? rc : grow(S, "gviol", (size_t)groups * 4, &d_gviol);
    if (rc) return rc;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t e = up(d_items, items.data(), items.size() * sizeof(qmc_item));
    if (e == hipSuccess) e = up(d_gbeg, gbeg.data(), (size_t)groups * 4);
    if (e == hipSuccess) e = up(d_gend, gend.data(), (size_t)groups * 4);
    if (e == hipSuccess) e = up(d_gdst, gdst.data(), (size_t)groups * 8);
    if (e == hipSuccess) e = up(d_gks, gks.data(), (size_t)groups * 4);
    for (const Launch &L : launches) {
        if (e != hipSuccess) break;
        const qmc_plan *P = L.plan;
        PlanPool &pp = S->pools[P];
        qmc_launch_args A{};
        A.sec = P->d_sec;
        A.lat = (const qmc_lat_dev *)pp.lat.p;
        A.texp = P->d_texp;
        A.texpd = P->d_texpd;
        A.tprog = P->d_tprog;
        A.toff = P->d_toff;
        A.dprog = P->d_dprog;
        A.tcoef = (const double *)pp.coef.p;
        A.dexp = P->d_dexp;
        A.dcoef = (const double *)pp.dcoef.p;
        A.shifts = (const double *)S->shift_pool.p;
        A.lam = (const double *)pp.lam.p;
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
        e = qmc_launch_serve_accumulate((const double *)d_partial, (const int32_t *)d_viol,
                                        (const int32_t *)d_gbeg, (const int32_t *)d_gend,
                                        (double *const *)d_gdst, (const int32_t *)d_gks, groups,
                                        kstride, (int32_t *)d_gviol, st);
    // the host arrays above are locals: the stream is drained below before
    // they go out of scope
    std::vector<int32_t> gviol(groups);
    if (e == hipSuccess && groups)
        e = hipMemcpyAsync(gviol.data(), d_gviol, (size_t)groups * 4, hipMemcpyDeviceToHost, st);
    // requests whose level completes in this step: combine their sums
    done_lv.clear();
    for (const Win &w : wins)
        if (w.end >= w.r->level_items) done_lv.push_back(w.r);
    std::vector<std::vector<double>> tots(done_lv.size());
    for (size_t i = 0; i < done_lv.size() && e == hipSuccess; ++i) {
        Request *r = done_lv[i];
        const qmc_plan *P = r->plan;
        const int K = P->tot_hi - P->tot_lo + 1;
        void *d_tot;
        char name[32];
        snprintf(name, sizeof name, "tot%zu", i);
        if (grow(S, name, (size_t)r->m * K * 16, &d_tot)) {
            e = hipErrorOutOfMemory;
            break;
        }
        e = qmc_launch_serve_combine((const double *)r->sums.p, P->d_sec,
                                     (const double *)S->pools[P].D.p, (int)P->secs.size(), r->m,
                                     P->kstride, K, P->tot_lo - P->c_lo,
                                     1.0 / (double)r->level_n,
                                     (double *)d_tot, st);
        tots[i].resize((size_t)r->m * K * 2);
        if (e == hipSuccess)
            e = hipMemcpyAsync(tots[i].data(), d_tot, tots[i].size() * 8, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return qmc_set_error(ctx, QMC_EDEVICE, "serving step: %s", hipGetErrorString(e));
    // bookkeeping
    for (const Win &w : wins) w.r->cursor = w.end;
    for (size_t g = 0; g < (size_t)groups; ++g) {
        Request *r = gown[g].first;
        r->level_viol += gviol[g];
        r->level_vsec[gown[g].second] += gviol[g];
    }
    for (size_t i = 0; i < done_lv.size(); ++i) {
        Request *r = done_lv[i];
        r->evals += r->level_count * (uint64_t)r->plan->secs.size() * r->m;
        r->steps += 1;
        if (r->level_viol > 0 && r->halvings_left > 0) {
            // back off lambda in the sectors concerned and restart at n0
            const int ns = (int)r->plan->secs.size();
            for (int s = 0; s < ns; ++s)
                if (r->level_vsec[s] > 0) r->lam[s] *= 0.5;
            r->halvings_left -= 1;
            r->halvings += 1;
            PlanPool &pp = S->pools[r->plan];
            hipError_t e2 = hipMemcpyAsync((char *)pp.lam.p + (size_t)r->slot * ns * 8,
                                           r->lam.data(), (size_t)ns * 8,
                                           hipMemcpyHostToDevice, st);
            if (e2 == hipSuccess)
                e2 = qmc_launch_fill((double *)r->sums.p, (long)(r->sums.bytes / 8), 0.0, st);
            if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
            if (e2 != hipSuccess)
                return qmc_set_error(ctx, QMC_EDEVICE, "serving: %s", hipGetErrorString(e2));
            r->n_cur = 0;
            r->coeff.assign(r->coeff.size(), qmc_coeff{});
            start_level(r);
            continue;
        }
        r->violations += r->level_viol;
        r->n_cur = r->level_n;
        assemble_totals(r->plan, r->m, tots[i], r->coeff);
    }
    return QMC_OK;
}

void scheduler(qmc_serve_state *S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    std::vector<Request *> done_lv;
    while (true) {
        S->cv.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->active.empty(); });
        if (S->stop) break;
        // cancellations
        for (auto it = S->active.begin(); it != S->active.end();) {
            if ((*it)->cancelled) {
                release_device(S, *it);
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
        // admission by slots and device memory: a request holds at most
        // request_bytes() beyond the plan pools while it is active
        while (!S->pending.empty() && (int)S->active.size() < S->ctx->max_slots) {
            Request *r = S->pending.front();
            // device memory outside serving, the pools, every active
            // request's bound and this one's (with its plan's pool if new)
            const int slots = S->ctx->max_slots;
            size_t more = request_bytes(r->plan, r->m, r->n0, r->n_max);
            if (!S->pools.count(r->plan)) more += plan_pool_bytes(r->plan, slots);
            if (!S->shift_pool.p) more += shift_pool_bytes(slots);
            const size_t used = S->ctx->used.load();
            const size_t other = used > S->pool_bytes ? used - S->pool_bytes : 0;
            const bool fits = other + S->fixed_bytes + S->admitted + more <= S->ctx->budget;
            int rc = QMC_OK;
            if (fits) {
                lk.unlock();
                rc = admit_device(S, r);
                lk.lock();
            }
            if (!fits || rc != QMC_OK) {
                if (r->slot >= 0) release_device(S, r);
                if (S->active.empty() || rc == QMC_EDEVICE) {   // cannot fit even alone
                    qmc_set_error(S->ctx, rc ? rc : QMC_EBUDGET,
                                  "request %llu does not fit the budget",
                                  (unsigned long long)r->ticket);
                    finish(S, r, rc ? rc : QMC_EBUDGET);
                    S->pending.pop_front();
                    continue;
                }
                break;
            }
            r->mem = request_bytes(r->plan, r->m, r->n0, r->n_max);
            S->admitted += r->mem;
            start_level(r);
            S->active.push_back(r);
            S->pending.pop_front();
        }
        S->done_cv.notify_all();
        if (S->active.empty()) continue;
        std::vector<Request *> act = S->active;
        lk.unlock();
        int rc = run_step(S, act, done_lv);
        lk.lock();
        if (rc == QMC_EBUDGET || rc == QMC_ENOMEM) {
            // the step buffers did not fit: retire the newest request only
            Request *r = S->active.back();
            release_device(S, r);
            qmc_set_error(S->ctx, rc, "request %llu retired: step buffers exceed the budget",
                          (unsigned long long)r->ticket);
            finish(S, r, rc);
            S->active.pop_back();
            S->done_cv.notify_all();
            continue;
        }
        for (auto it = S->active.begin(); it != S->active.end();) {
            Request *r = *it;
            bool retire = false;
            const bool level_done =
                std::find(done_lv.begin(), done_lv.end(), r) != done_lv.end();
            if (rc != QMC_OK) {
                finish(S, r, rc);
                retire = true;
            } else if (level_done && r->n_cur != 0) {
                if (r->violations > 0) {
                    finish(S, r, QMC_EDEFORM);
                    retire = true;
                } else if (converged(r)) {
                    finish(S, r, QMC_OK);
                    retire = true;
                } else if (2 * r->n_cur > r->n_max) {
                    finish(S, r, QMC_ENOTCONVERGED);
                    retire = true;
                } else {
                    start_level(r);
                }
            }
            if (retire) release_device(S, r);
            it = retire ? S->active.erase(it) : it + 1;
        }
        S->done_cv.notify_all();
    }
    // drain
    for (Request *r : S->active) {
        release_device(S, r);
        finish(S, r, QMC_ECANCELLED);
    }
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
    for (auto &kv : S->bufs) dev_free(S, kv.second);
    dev_free(S, S->shift_pool);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    ctx->serve = nullptr;
}

extern "C" int qmc_submit(qmc_ctx *ctx, const qmc_plan *plan, const qmc_request *req,
                          uint64_t *ticket)
{
    if (!ctx || !plan || !req || !ticket || !req->kin || !req->z)
        return qmc_set_error(ctx, QMC_EINVAL, "null argument");
    if (req->m < 2 || req->m > MAX_SHIFTS)
        return qmc_set_error(ctx, QMC_EINVAL, "need 2 <= m <= %d shifts", MAX_SHIFTS);
    auto pow2 = [](uint64_t v) { return v >= 2 && (v & (v - 1)) == 0; };
    if (!pow2(req->n0) || !pow2(req->n_max) || req->n0 > req->n_max ||
        req->n_max >= (1ull << 31))
        return qmc_set_error(ctx, QMC_EINVAL, "n0 <= n_max must be powers of two below 2^31");
    if (!(req->rel_err_target > 0.0))
        return qmc_set_error(ctx, QMC_EINVAL, "rel_err_target must be positive");
    if (plan->opts.precision == QMC_FP32_EVAL && req->rel_err_target < QMC_FP32_TARGET_FLOOR)
        return qmc_set_error(ctx, QMC_EINVAL,
                             "FP32-eval plans: rel_err_target must be >= %g (rounding bias)",
                             QMC_FP32_TARGET_FLOOR);
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
