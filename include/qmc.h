/*
 * qmc.h -- C ABI of libqmc: quasi-Monte Carlo integration of
 * sector-decomposed Feynman-parameter integrals on one AMD Instinct
 * MI355X (gfx950).
 *
 * Method (Li, Wang, Yan, Zhao, "Efficient Numerical Evaluation of Feynman
 * Integrals", Chin. Phys. C 40 (2016) 033103):
 *   - the integral is given as a list of sectors, each of the form of
 *     Eq. 9 (Section II): a monomial prod_j t_j^(a_j + b_j eps) times powers
 *     U(t)^(u0 + u1 eps) F(t)^(f0 + f1 eps) of two polynomials whose
 *     constant terms do not vanish, times a constant D;
 *   - poles t^(-1 + b eps) are subtracted as in Eq. 11 and the integrand is
 *     expanded in eps;
 *   - in the physical region the contour is deformed as in Eq. 14,
 *     z_j = t_j - i lambda t_j (1 - t_j) dF/dt_j;
 *   - every sector is integrated with the shifted rank-1 lattice rule of
 *     Section III (Eqs. 17-18) after a Korobov periodising transform (Eq. 21
 *     generalised to order r); the mean over the m shifts is the estimate
 *     (Eq. 19) and their spread gives the error (Eq. 20).
 *
 * Conventions
 *   - All functions return int: QMC_OK (0) on success, QMC_PENDING (> 0)
 *     where noted, a negative QMC_E* code on failure; qmc_last_error(ctx)
 *     then holds a message (per context, overwritten by the next error).
 *   - Every input pointer is caller-owned host memory, read during the call
 *     (copied or uploaded) and not retained.  Every output pointer is
 *     caller-allocated host memory of the stated size.
 *   - Device memory is allocated by the library (hipMalloc) and counted
 *     against the context's HBM budget.  Plans are immutable after creation.
 *   - A context is bound to one device and one HIP stream; calls on one
 *     context must not overlap, except qmc_submit / qmc_poll / qmc_wait /
 *     qmc_cancel, which are thread-safe.
 *   - Complex numbers are stored as (re, im) pairs of doubles.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define QMC_OK 0
#define QMC_PENDING 1            /* request still running (qmc_poll/qmc_wait) */
#define QMC_EINVAL (-1)          /* bad sizes, exponents, missing constant term, m < 2 */
#define QMC_EUNREGULATED (-2)    /* a_j = -1 with b_j = 0 (pole not regulated), also when
                                    reached by integration by parts */
#define QMC_EUNSUPPORTED (-3)    /* too many poles, orders or numerator factors, dim >
                                    QMC_MAX_DIM, integration by parts with lambda > 0 */
#define QMC_ENOMEM (-4)          /* host or device allocation failed */
#define QMC_EBUDGET (-5)         /* request does not fit the HBM budget */
#define QMC_EDEFORM (-6)         /* Im F(z) > 0, Re U(z) <= 0 or F <= 0 without deformation */
#define QMC_ENOTCONVERGED (-7)   /* n_max reached before the error target */
#define QMC_EDEVICE (-8)         /* HIP runtime error */
#define QMC_ECANCELLED (-9)      /* request cancelled */

/* ---- limits -------------------------------------------------------------- */
#define QMC_MAX_DIM 8            /* integration variables per sector */
#define QMC_MAX_POLES 4          /* variables with a_j = -1 per sector */
#define QMC_MAX_ORDERS 8         /* Laurent orders carried per sector */
#define QMC_MAX_FACTORS 4        /* numerator factors per sector after Eq. 13 */
#define QMC_MAX_EXP 15           /* largest exponent of a polynomial term */

/* ---- pole methods (qmc_plan_opts.pole_method) ---------------------------- */
#define QMC_POLES_SUBTRACT 0     /* poles a_j = -1 subtracted (Eq. 11) */
#define QMC_POLES_IBP 1          /* poles a_j = -1 integrated by parts (Eq. 13) as well */

/* ---- precision modes ----------------------------------------------------- */
#define QMC_FP64 0               /* all arithmetic in FP64 */
#define QMC_FP32_EVAL 1          /* FP32 integrand, FP64 where stability needs it */
/* FP32_EVAL: periodiser, monomials, U and F, the Moebius algebra and the
 * eps series of Euclidean sectors in FP32; for deformed sectors the power
 * table, derivative terms, z and the complex monomials of U(z), F(z) in
 * FP32, the Jacobian determinant and the logarithms/powers of U and F in
 * FP64; lattice points, corner differences and all sums in FP64.  The
 * Eq. 20 error does not include the FP32 rounding bias (measured up to
 * 3.2e-6 relative on the double box); serving requests on FP32_EVAL plans
 * must ask for rel_err_target >= QMC_FP32_TARGET_FLOOR. */
#define QMC_FP32_TARGET_FLOOR 1e-5

typedef struct qmc_ctx qmc_ctx;     /* device, stream, budget, scheduler */
typedef struct qmc_plan qmc_plan;   /* device-resident sector tables */
typedef struct qmc_job qmc_job;     /* one bound integration (inputs resident) */

/* Sparse polynomial sum_a c_a prod_j t_j^exps[a][j].  Its coefficients are
 * linear in the kinematic invariants: c_a = sum_k coef[a][k] * kin[k], with
 * kin[0] = 1 (Section II: U and F are linear in the invariants and masses). */
typedef struct {
    int32_t n_terms;
    const uint8_t *exps;         /* [n_terms][dim], each <= QMC_MAX_EXP */
    const double *coef;          /* [n_terms][n_inv] */
} qmc_poly;

/* One sector (Eq. 9): D * prod_j t_j^(a_j + b_j eps) U^(u0 + u1 eps) F^(f0 + f1 eps).
 * a_j = -1 (then b_j != 0): the pole is subtracted (Eq. 11), or, with
 * pole_method QMC_POLES_IBP, integrated by parts (Eq. 13).  a_j < -1 (as
 * dotted propagators give): the plan applies the integration by parts of
 * Eq. 13 in that variable until its power is -1 or above -1 (with
 * QMC_POLES_IBP: above -1), which turns the sector into several, with
 * numerator factors (derivatives of U and F) and an eps-dependent
 * coefficient each; Euclidean plans only (lambda = 0).
 * U and F must contain the all-zero exponent (their constant term). */
typedef struct {
    int32_t dim;                 /* 1 .. QMC_MAX_DIM */
    const double *mono_a;        /* [dim] */
    const double *mono_b;        /* [dim] */
    qmc_poly U, F;
    double u_exp[2];             /* u0, u1 */
    double f_exp[2];             /* f0, f1 */
    double coef_re, coef_im;     /* D */
} qmc_sector;

/* The whole integral: sum over sectors, times a prefactor series (e.g. the
 * Gamma function of Eq. 5), Laurent orders eps_lo .. eps_hi returned. */
typedef struct {
    int32_t n_sectors;
    const qmc_sector *sectors;
    int32_t n_inv;               /* invariants per kinematic point, kin[0] = 1 */
    int32_t eps_lo, eps_hi;
    const double *prefactor;     /* [n_pref][2]: coefficients of eps^(eps_pref_lo + q) */
    int32_t eps_pref_lo, n_pref;
} qmc_problem;

typedef struct {
    int32_t precision;           /* QMC_FP64 or QMC_FP32_EVAL */
    int32_t korobov_r;           /* periodiser order 0..3 (Eq. 21 is r = 1) */
    double lambda;               /* deformation parameter; 0 = Euclidean */
    int32_t points_per_lane;     /* 0 = chosen by the library */
    int32_t pole_method;         /* QMC_POLES_SUBTRACT or QMC_POLES_IBP */
} qmc_plan_opts;

/* Rank-1 lattice (Eq. 17): points {i z / n}, i = 0 .. n-1; 2 <= n < 2^31,
 * z[j] coprime to n.  z has QMC_MAX_DIM entries; a sector of dimension d
 * uses z[0..d-1]. */
typedef struct {
    uint64_t n;
    const uint32_t *z;
} qmc_lattice;

typedef struct { double re, im, err_re, err_im; } qmc_coeff;

/* Per-plan facts for callers laying out optional outputs. */
typedef struct {
    int32_t n_sectors, n_inv;
    int32_t sec_lo, sec_orders;  /* sector Laurent orders sec_lo .. sec_lo+sec_orders-1 */
    int32_t eps_lo, eps_hi;
    int32_t max_poles, deform;
    double flops_per_point;      /* algorithmic FP64 flops of one lattice point, summed over sectors */
    int32_t n_input_sectors;     /* sectors given; n_sectors counts them after Eq. 13 */
    int32_t max_factors;         /* most numerator factors of a sector (Eq. 13) */
} qmc_plan_info;

/* One planned sector, as the integration by parts of Eq. 13 left it:
 *   C(eps) * prod_j t_j^(a_j + b_j eps) * P_1 .. P_r * U^(u0 + u1 eps) F^(f0 + f1 eps)
 * over `dim` variables (the input sector's, minus those set to 1 by
 * boundary terms; 1 dummy variable if none is left).  Planned sectors come
 * in a fixed order: input sectors in order; within one, its variables in
 * increasing index, each application of Eq. 13 giving the boundary term,
 * then the derivative terms (numerator factors in order, then U, then F),
 * each expanded completely before the next.  A sector without exponents
 * below -1 (with QMC_POLES_IBP: without exponents <= -1) is planned
 * unchanged (C = D, no factor).  With QMC_POLES_IBP every pole a_j = -1
 * contributes 1/(b_j eps) to C, so C starts at eps^-p (p poles taken) and
 * the planned sector has no pole left. */
typedef struct {
    int32_t origin;              /* index of the input sector */
    int32_t dim;                 /* integration variables */
    int32_t poles;               /* variables with a_j = -1 (Eq. 11) */
    int32_t factors;             /* numerator factors r */
    double u_exp[2], f_exp[2];   /* powers of U and F */
    double coef[QMC_MAX_ORDERS][2];   /* C(eps) = sum_k coef[k] eps^(coef_lo + k) (re, im) */
    int32_t coef_lo;             /* 0, or -QMC_MAX_POLES with QMC_POLES_IBP */
} qmc_sector_info;

typedef struct {
    qmc_coeff *coeff;            /* [n_points][eps_hi-eps_lo+1] */
    double *per_shift;           /* optional [n_points][m][eps_hi-eps_lo+1][2] */
    double *sector_sums;         /* optional [n_points][n_sectors][m][sec_orders][2]:
                                    raw sums sum_i w g (no 1/n, no D) */
    uint64_t evals;              /* integrand evaluations (points x sectors x shifts) */
    uint64_t n_final;            /* lattice size of the final iteration (serving) */
    int32_t status;              /* QMC_OK, QMC_EDEFORM, ... */
    int32_t deform_violations;   /* points with Im F(z) > 0 or Re U(z) <= 0 */
    double kernel_ms;            /* device time of the integrand kernels */
    double algo_flops;           /* algorithmic flops of the integrand kernels */
    double latency_ms;           /* serving: submit to completion (0 for qmc_integrate) */
    int32_t steps;               /* serving: lattice sizes evaluated (doublings + 1) */
    int32_t lambda_halvings;     /* serving: deformation back-offs taken (see qmc_request) */
} qmc_result;

/* Create a context on `device` with at most hbm_budget bytes of device
 * memory (0 = 64 GiB) and at most max_slots concurrent serving requests
 * (0 = 64).  Creates a HIP stream of default priority. */
int qmc_create(int device, size_t hbm_budget, int max_slots, qmc_ctx **out);
void qmc_destroy(qmc_ctx *ctx);
/* Use a caller-owned stream (e.g. PyTorch's current stream) instead. */
int qmc_set_stream(qmc_ctx *ctx, void *hip_stream);
const char *qmc_last_error(qmc_ctx *ctx);

/* Plan the sectors of Eq. 9 (Section II): validate them, apply Eq. 13
 * where some a_j < -1 (with QMC_POLES_IBP: a_j <= -1), permute each
 * sector's variables so the subtracted ones come first, sort polynomial
 * terms by which of those they contain, derive dF and d2F tables when
 * lambda > 0, and upload the tables.  Everything sized "per sector" below
 * (lat_per_sector, sector_sums, qmc_size_lattices) counts planned sectors,
 * qmc_plan_info.n_sectors of them. */
int qmc_plan_sectors(qmc_ctx *ctx, const qmc_problem *problem,
                     const qmc_plan_opts *opts, qmc_plan **out);
void qmc_plan_free(qmc_plan *plan);
int qmc_plan_get_info(const qmc_plan *plan, qmc_plan_info *info);
/* Planned sector s (0 <= s < n_sectors); QMC_EINVAL if out of range. */
int qmc_plan_sector_info(const qmc_plan *plan, int32_t s, qmc_sector_info *out);

/* Integrate at n_points kinematic points kin[n_points][n_inv] with the
 * lattice `lat` (or lat_per_sector[n_sectors] if not NULL) and the shifts
 * shifts[m][QMC_MAX_DIM] (m >= 2): the shifted rank-1 lattice sums of
 * Section III (Eqs. 17-18, Korobov periodiser Eq. 21 at order korobov_r)
 * of every sector's subtracted integrand (Eqs. 9-11; Eq. 14 when
 * lambda > 0), combined per shift into the Laurent coefficients and
 * reduced to mean and error (Eqs. 19-20).  Blocks until the result is
 * ready. */
int qmc_integrate(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                  int32_t n_points, const qmc_lattice *lat,
                  const qmc_lattice *lat_per_sector, const double *shifts,
                  int32_t m, qmc_result *out);

/* Per-sector lattice sizes for a total budget of lattice points (uneven
 * sizing across sectors, the sizing of Section III's error estimate applied
 * per sector).  A pilot integration at the kinematic point kin[n_inv] on
 * the lattice `pilot` with shifts[m][QMC_MAX_DIM] gives each sector's spread
 * c_s over the shifts (largest over orders and real/imaginary parts of
 * |S_k/n - mean_k S_k/n|).  With a lattice error ~ c_s / n_s and a cost
 * proportional to the sector's algorithmic flops f_s per point, minimising
 * sum_s (c_s / n_s)^2 at fixed sum_s f_s n_s gives n_s ~ (c_s^2 / f_s)^(1/3);
 * the sizes are scaled so that sum_s n_s = total_points and each is rounded,
 * in log scale, to the nearest of sizes[n_sizes] (the caller's lattices).
 * out_n[n_sectors] receives the chosen sizes.  Errors: QMC_EINVAL on bad
 * sizes or pointers; those of qmc_integrate for the pilot. */
int qmc_size_lattices(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                      const qmc_lattice *pilot, const double *shifts, int32_t m,
                      uint64_t total_points, const uint64_t *sizes, int32_t n_sizes,
                      uint64_t *out_n);

/* ---- allocation-free variant ------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * qmc_integrate_noalloc computes exactly what qmc_integrate computes (same
 * kernels, work list and summation order, hence the same bits), but every
 * device buffer of the call lives in one fixed device array of
 * QMC_NOALLOC_SCRATCH_BYTES that the library reserves on each device it is
 * loaded on and keeps until the process ends; the call makes no device or
 * pinned-host allocation (host-side planning still uses the C++ heap).
 * Sizes: the call needs about 200 bytes per work item (items are tiles of
 * 256 x points-per-lane lattice indices of one point, sector and shift) plus
 * the contracted coefficients; a call that needs more than the array
 * returns QMC_EBUDGET with the size it needed and runs nothing.  Every call
 * on a device shares that device's array: calls on one device are
 * serialised by the library and each waits for its stream to drain before
 * it returns, so overlapping calls from several host threads are safe but
 * run one after another.  kernel_ms is reported as 0.  Errors as for
 * qmc_integrate. */
#define QMC_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int qmc_integrate_noalloc(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                          int32_t n_points, const qmc_lattice *lat,
                          const qmc_lattice *lat_per_sector, const double *shifts,
                          int32_t m, qmc_result *out);

/* The same in three steps: bind uploads the inputs and allocates device
 * outputs; run enqueues the kernels on the context stream (asynchronous);
 * fetch waits for them, copies the per-shift sums back and assembles. */
int qmc_bind(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
             int32_t n_points, const qmc_lattice *lat,
             const qmc_lattice *lat_per_sector, const double *shifts,
             int32_t m, qmc_job **out);
int qmc_run(qmc_job *job);
int qmc_fetch(qmc_job *job, qmc_result *out);
void qmc_job_free(qmc_job *job);

/* ---- batching: graph replay and autotuning ---------------------------------
 * qmc_job_set_graph: when enabled, the next qmc_run captures the job's whole
 * launch sequence (integrand kernels of every class, the reduction, the copy
 * of the group sums) into one HIP graph and later runs replay it.  The
 * timing in qmc_result.kernel_ms then covers the whole graph.
 *
 * qmc_autotune: times candidate launch shapes on the given inputs (which
 * should have the lattice sizes of the production runs; two shifts are
 * enough) and remembers, per (plan, poles, kernel width, lattice-size
 * octave), the fastest points per lane (the length of each lane's point
 * loop), persistent-grid setting and occupancy build (waves per SIMD); a
 * shape later in the order of preference (points per lane 64, 16, 256, 4,
 * 1024; then build 0, 1; then grid off, 4, 8 per CU) must be more than 2%
 * faster to replace an earlier one, so noise does not flip choices.  Later
 * binds with points_per_lane = 0 use them.  choices (may be NULL) receives
 * up to max_choices entries; *n_choices is set to the number of classes. */
typedef struct {
    int32_t poles, width;        /* kernel class: poles, complex width (0 = real) */
    int32_t points_per_lane;     /* chosen tile: 256 * points_per_lane indices per item */
    int32_t grid_per_cu;         /* 0: one work-group per item; else persistent */
    int32_t occupancy_variant;   /* 0: build with the swept waves per SIMD; 1: the build
                                    with fewer waves (real kernels one fewer, deformed 2) */
    int32_t pad;
    double ms;                   /* measured time of the class with that shape */
} qmc_tune_choice;

int qmc_job_set_graph(qmc_job *job, int enable);

/* Run every kernel class of a bound job with occupancy build `variant`
 * (0 or 1, as qmc_tune_choice.occupancy_variant) instead of the one the
 * bind chose; a captured graph is dropped and captured again on the next
 * run.  Both builds compute the same sums (to rounding).  QMC_EINVAL for
 * another variant or while the job is running. */
int qmc_job_set_variant(qmc_job *job, int32_t variant);

/* Per-kernel accounting of a bound job.  Each class of work items (poles,
 * complex width) is one kernel launch per qmc_run.  qmc_job_set_profiling
 * with enable != 0 records a HIP event pair around every class launch of
 * later eager runs (not inside a graph); qmc_job_class_stats copies up to
 * max entries, one per class in launch order, and sets *n to the number of
 * classes.  ms is the event time of that launch in the last completed eager
 * run (after qmc_fetch), -1 when it was not timed.  algo_flops counts the
 * algorithmic FP64 (or FP32) operations of the launch with the convention
 * add/mul 1, fma 2, division and log/exp 20 per lattice point of Eq. 16's
 * inner sum, summed over the launch's points.  Errors: QMC_EINVAL on a null
 * job or n. */
typedef struct {
    int32_t poles, width;        /* class: poles, complex width (0 = real) */
    int32_t points_per_lane;     /* tile of one item is 256 * points_per_lane */
    int32_t grid;                /* work-groups launched */
    int32_t items;               /* work items in the class */
    int32_t precision;           /* QMC_FP64 or QMC_FP32_EVAL */
    uint64_t evals;              /* integrand evaluations of one launch */
    double algo_flops;           /* algorithmic flops of one launch */
    double ms;                   /* launch time of the last eager run, or -1 */
    int32_t variant;             /* occupancy build launched (see qmc_tune_choice) */
    int32_t pad;
} qmc_class_stat;

int qmc_job_set_profiling(qmc_job *job, int enable);
int qmc_job_class_stats(const qmc_job *job, qmc_class_stat *out, int32_t max, int32_t *n);

int qmc_autotune(qmc_ctx *ctx, const qmc_plan *plan, const double *kin, int32_t n_points,
                 const qmc_lattice *lat, const qmc_lattice *lat_per_sector,
                 const double *shifts, int32_t m, qmc_tune_choice *choices,
                 int32_t max_choices, int32_t *n_choices);

/* ---- diagnostics -------------------------------------------------------------
 * qmc_math_eval applies one of the elementary functions that the integrand
 * kernels use for the logarithms of Eq. 9's factors, the monomials of U and
 * F and the eps expansion (fn: QMC_MATH_LN for x > 0, QMC_MATH_LN1P for
 * x > -1, QMC_MATH_EXP and QMC_MATH_EXPM1 for finite x, QMC_MATH_RCP, the
 * reciprocal of the divisions, for normal x; the _F32 codes: the float
 * versions of FP32 evaluation, applied to x rounded to float) to n doubles x
 * (device) and writes y (device, n doubles) on the context stream, then
 * waits for it.  Outside those domains the result is unspecified.  For tests
 * that bound their error.  Errors: QMC_EINVAL (null pointer, n < 0, unknown
 * fn), QMC_EDEVICE. */
enum { QMC_MATH_LN = 0, QMC_MATH_LN1P = 1, QMC_MATH_EXP = 2, QMC_MATH_EXPM1 = 3, QMC_MATH_RCP = 4,
       QMC_MATH_LN_F32 = 5, QMC_MATH_LN1P_F32 = 6, QMC_MATH_EXP_F32 = 7,
       QMC_MATH_EXPM1_F32 = 8 };
int qmc_math_eval(qmc_ctx *ctx, int32_t fn, const double *x, double *y, int64_t n);

/* ---- serving (continuous batching) ---------------------------------------
 * A request is one integral (a plan) at one kinematic point with a relative
 * error target.  A scheduler thread owned by the context admits requests
 * while fewer than max_slots are active and their device memory fits the
 * HBM budget, and repeatedly launches one batch that advances every active
 * request by one lattice size: n0 first, then n -> 2n evaluating only the
 * new (odd) indices of the embedded rank-1 lattice {i z / 2n} (Eq. 17),
 * whose even indices are the previous lattice.  Per-shift sums stay
 * resident per request; after each batch the result (Eqs. 19-20) is
 * checked against the target, and the request completes when every order
 * has err/|mean| <= target (orders below 1e-3 of the largest are compared
 * absolutely against the largest), when n_max is reached
 * (QMC_ENOTCONVERGED), or when it is cancelled.  If a batch finds points
 * where the deformed contour violates the sign conditions (Im F(z) > 0 or
 * Re U(z) <= 0; Eq. 14 guarantees them only for small enough lambda), the
 * request retires with QMC_EDEFORM unless it still has back-offs
 * (lambda_halvings): then lambda is halved in the sectors that violated
 * and the request restarts at n0 with its sums cleared.  A sector's
 * integral does not depend on the contour (Cauchy), so only its variance
 * changes.  A request's arithmetic does
 * not depend on the other requests in the batch, so its result is the
 * same alone and in the mix. */
typedef struct {
    const double *kin;           /* [n_inv] one kinematic point */
    double rel_err_target;       /* stop when err/|mean| <= target for every order */
    uint64_t n0, n_max;          /* embedded lattice sizes (powers of two, n_max < 2^31) */
    int32_t m;                   /* shifts (>= 2) */
    uint64_t seed;               /* SplitMix64 seed of the shifts (k-major, 53-bit) */
    const uint32_t *z;           /* [QMC_MAX_DIM] odd generating vector */
    int32_t lambda_halvings;     /* deformed sectors: back-offs allowed (0..16), see below */
    int32_t pad;
} qmc_request;

/* Queue a request; returns a ticket.  Thread-safe; returns immediately. */
int qmc_submit(qmc_ctx *ctx, const qmc_plan *plan, const qmc_request *req,
               uint64_t *ticket);
/* QMC_PENDING while the request runs; its status code when done (the
 * result is filled, out->coeff sized as for qmc_integrate with one point). */
int qmc_poll(qmc_ctx *ctx, uint64_t ticket, qmc_result *out);
/* Block until done or timeout_s elapses (< 0: no timeout). */
int qmc_wait(qmc_ctx *ctx, uint64_t ticket, double timeout_s, qmc_result *out);
/* Cancel a queued or running request (it completes with QMC_ECANCELLED). */
int qmc_cancel(qmc_ctx *ctx, uint64_t ticket);
/* Release the bookkeeping of a finished request. */
int qmc_release(qmc_ctx *ctx, uint64_t ticket);

#ifdef __cplusplus
}
#endif
#endif /* QMC_H */
