// Host-side state of libqmc (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qmc.h"
#include "qmc_device.h"
#include "qmc_kernels.h"

struct qmc_serve_state;

static_assert(QMC_NFMAX == QMC_MAX_FACTORS, "numerator factor limits differ");
static_assert(QMC_NCOEF == QMC_MAX_ORDERS, "coefficient series lengths differ");

// Launch shape chosen by the autotuner for one kernel class.
struct qmc_tune {
    int ppl = 0;                     // points per lane per work item
    int grid_per_cu = 0;             // persistent work-groups per CU (0: one per item)
    int variant = 0;                 // occupancy build of the kernel class
    double ms = 0.0;                 // measured time of the class
};


struct qmc_ctx {
    int device = 0;
    size_t budget = 0;
    std::atomic<size_t> used{0};
    int max_slots = 64;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    std::mutex err_mu;
    std::string last_error;
    qmc_serve_state *serve = nullptr;
    std::mutex serve_mu;
    int n_cu = 256;                  // compute units of the device
    std::mutex tune_mu;
    std::map<std::string, qmc_tune> tuned;   // autotuner results by class key
};

// An input sector after the integration by parts of Eq. 13 (qmc_ibp.cpp),
// or unchanged when none of its exponents is below -1: exponents, U, F and
// numerator factors as term lists ([terms][dim] exponents, [terms][n_inv]
// coefficients), powers of U and F, and the coefficient series C(eps)
// (eps^0 .. QMC_MAX_ORDERS-1, times the input sector's D).
struct qmc_ibp_sec {
    int origin = 0;                  // index of the input sector
    int dim = 0;
    bool ibp = false;                // Eq. 13 was applied to the input sector
    std::vector<double> a, b;
    std::vector<uint8_t> eU, eF;
    std::vector<double> cU, cF;
    std::vector<std::vector<uint8_t>> eP;
    std::vector<std::vector<double>> cP;
    double u0 = 0, u1 = 0, f0 = 0, f1 = 0;
    std::vector<std::complex<double>> C;  // C[e]: coefficient of eps^(clo + e)
    int clo = 0;
};

// Every sector of the problem expanded by Eq. 13 where needed (powers below
// -1; with `poles`, powers -1 as well), in the documented order.  Returns
// QMC_OK or an error code with a message in err.
int qmc_ibp_expand(const qmc_problem *pb, bool poles, std::vector<qmc_ibp_sec> &out,
                   char *err, size_t errlen);

// One sector as planned: permuted exponents, term ranges, flop count.
struct qmc_sec_host {
    int dim = 0, ks = 0, K = 0, deform = 0;
    int perm[QMC_DMAX] = {};
    double a[QMC_DMAX] = {}, b[QMC_DMAX] = {}, inv_b[QMC_DMAX] = {};
    int aint[QMC_DMAX] = {};
    int32_t um[QMC_NMASK + 1] = {}, fm[QMC_NMASK + 1] = {};
    int32_t um1[QMC_NMASK] = {}, um2[QMC_NMASK] = {};
    int32_t fm1[QMC_NMASK] = {}, fm2[QMC_NMASK] = {};
    int32_t d1[QMC_DMAX + 1] = {};
    int32_t d2[QMC_DMAX * (QMC_DMAX + 1) / 2 + 1] = {};
    double u0 = 0, u1 = 0, f0 = 0, f1 = 0;
    int u0i = 0, f0i = 0;
    double lambda = 0.0;
    bool mono_log = false;       // some term needs exp(sum_j e_j ln t_j)
    int origin = 0;                  // input sector it comes from
    int nf = 0;                      // numerator factors (Eq. 13)
    int32_t pm[QMC_NFMAX][QMC_NMASK + 1] = {};
    int32_t pm1[QMC_NFMAX][QMC_NMASK] = {}, pm2[QMC_NFMAX][QMC_NMASK] = {};
    std::vector<std::complex<double>> C{1.0};   // coefficient series, eps^c_lo ..
    std::vector<int> term_nnz;   // non-zero exponents per term (U and F)
    std::vector<int> dterm_nnz;  // the same for the derivative terms
    double flops = 0.0;          // algorithmic flops per lattice point
    double flops_deform = 0.0;   // the same on a deformed contour
    qmc_sec_dev dev() const;
};

struct qmc_plan {
    qmc_ctx *ctx = nullptr;
    uint64_t id = 0;                 // unique per process: keys the autotuner's choices
    qmc_plan_opts opts{};
    int n_inv = 0;
    int eps_lo = 0, eps_hi = 0, eps_pref_lo = 0, n_pref = 0;
    std::vector<double> pref;        // [n_pref][2]
    int sec_lo = 0, sec_hi = 0;      // sector orders carried
    int tot_lo = 0, tot_hi = 0;      // orders of sum_s C_s(eps) I_s(eps)
    int c_lo = 0;                    // order of C[0] in every sector's series C
    int kb = 1;                      // orders from eps^0 up: sec_hi + 1
    int kstride = 1;                 // order slots per group: kb + max_ks
    int max_ks = 0;
    int n_input_sectors = 0;         // sectors given; secs holds them after Eq. 13
    std::vector<qmc_sec_host> secs;
    std::vector<uint32_t> texp;      // packed exponents of all U and F terms
    std::vector<double> tcoef_rows;  // [n_terms][n_inv]
    std::vector<uint32_t> dexp;      // packed exponents of derivative terms
    std::vector<double> dcoef_rows;  // [n_dterms][n_inv]
    int n_terms = 0;
    double flops_per_point = 0.0;
    qmc_sec_dev *d_sec = nullptr;
    uint32_t *d_texp = nullptr;
    double *d_texpd = nullptr;
    uint32_t *d_tprog = nullptr;
    uint32_t *d_toff = nullptr;      // [2][n_terms][4] power-table byte offsets
    uint32_t *d_dprog = nullptr;
    uint32_t *d_dexp = nullptr;
};

// Kernel build of sector s: 1 = with numerator factors (Eq. 13).  The
// builds without them carry at most 3 orders above the poles; wider
// sectors (Eq. 13 taken at the poles) use the numerator build, where no
// factor is a product of 1.
inline int qmc_num_class(const qmc_plan *P, int s)
{
    return P->secs[s].nf > 0 || P->kb > 3 ? 1 : 0;
}

// largest grid of one launch: (2^32 - 1) work-items / QMC_BLOCK lanes
constexpr int QMC_MAX_GRID = (int)(0xffffffffu / QMC_BLOCK);

struct qmc_class {                   // items launched by one kernel instance
    int ks = 0, kb = 1, deform = 0, dm = 0;
    int num = 0;                     // sectors with numerator factors (Eq. 13)
    int begin = 0, end = 0;
    int grid = 0;                    // work-groups (0: one per item)
    int ppl = 0;                     // lattice points per lane per item
    int variant = 0;                 // occupancy build (0 swept default, 1 fewer waves)
    uint64_t evals = 0;              // integrand evaluations of one launch
    double flops = 0.0;              // algorithmic flops of one launch
};


int qmc_class_grid(const qmc_class &c);

struct qmc_job {
    qmc_ctx *ctx = nullptr;
    const qmc_plan *plan = nullptr;
    int n_points = 0, m = 0, ppl = 0;
    int n_items = 0, n_groups = 0;
    uint64_t evals = 0;
    std::vector<uint64_t> n_per_sector;
    std::vector<qmc_class> classes;
    std::vector<std::pair<void *, size_t>> bufs;
    qmc_lat_dev *d_lat = nullptr;
    double *d_coef = nullptr, *d_dcoef = nullptr, *d_shift = nullptr, *d_lam = nullptr;
    qmc_item *d_items = nullptr;
    int32_t *d_gbeg = nullptr, *d_gend = nullptr;
    double *d_partial = nullptr, *d_out = nullptr;
    int32_t *d_viol = nullptr, *d_gviol = nullptr;
    double *h_out = nullptr;         // pinned copies of the group sums
    int32_t *h_gviol = nullptr;
    size_t h_out_n = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> ev_cls;  // per-class timing (autotuner, profiling)
    bool cls_timed = false;          // the last run recorded ev_cls
    std::vector<double> cls_ms;      // per-class times of the last fetched run
    bool launched = false;
    bool use_graph = false;
    hipGraphExec_t graph = nullptr;
};

// Host arrays of a bound job's device inputs (filled by qmc_job_prepare).
struct qmc_job_host {
    std::vector<qmc_lat_dev> lats;   // [n_sectors]
    std::vector<double> coef, dcoef; // [n_points][n_terms], [n_points][n_dterms]
    std::vector<double> lam;         // [n_points][n_sectors]
    std::vector<qmc_item> items;
    std::vector<int32_t> gbeg, gend; // [n_groups]
    const double *shifts = nullptr;  // caller's [m][QMC_DMAX]
};

int qmc_job_prepare(qmc_ctx *ctx, const qmc_plan *plan, const double *kin, int32_t n_points,
                    const qmc_lattice *lat, const qmc_lattice *lat_per_sector,
                    const double *shifts, int32_t m, int ppl_override, int grid_override,
                    qmc_job *job, qmc_job_host &H);
hipError_t qmc_enqueue(qmc_job *job, bool timing);
int qmc_result_fill(qmc_job *job, const double *gsum, const int32_t *gviol, qmc_result *out);
int qmc_dev_alloc(qmc_ctx *ctx, void **p, size_t bytes);
void qmc_dev_free(qmc_ctx *ctx, void *p, size_t bytes);
int qmc_bind_impl(qmc_ctx *ctx, const qmc_plan *plan, const double *kin, int32_t n_points,
                  const qmc_lattice *lat, const qmc_lattice *lat_per_sector,
                  const double *shifts, int32_t m, int ppl_override, int grid_override,
                  bool class_timing, qmc_job **out);
std::string qmc_tune_key(const qmc_plan *plan, int ks, int dm, int num, uint64_t n);
void qmc_job_release(qmc_job *job);
int qmc_assemble(const qmc_plan *plan, int n_points, int m, const std::vector<uint64_t> &nsec,
                 const double *gsum, qmc_result *out);
void qmc_serve_shutdown(qmc_ctx *ctx);
void qmc_contract(const qmc_plan *plan, const double *kin, double *coef, double *dcoef);
int qmc_sector_mode(const qmc_plan *plan, int s, const double *coef, double *lam);
hipError_t qmc_launch_class(const qmc_plan *plan, const qmc_class &c, const qmc_launch_args &A,
                            hipStream_t stream);
int qmc_set_error(qmc_ctx *ctx, int code, const char *fmt, ...);
// Looks up the device address of the allocation-free entry point's scratch
// array on `device` (which must be current); called once per context.
int qmc_noalloc_setup(int device);
