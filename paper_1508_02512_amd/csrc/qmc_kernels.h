// Host-side launchers of the integrand and reduction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_device.h"

// Real (Euclidean) integrand for sectors with `ks` poles carrying ks + kb
// Laurent orders, evaluated in FP64 or FP32; one work-group per item in
// [item_begin, item_end).  variant 0 is the build with the swept occupancy,
// variant 1 the build with one wave per SIMD fewer (less spilling).  num:
// the sectors carry numerator factors (Eq. 13; variant 0 only); only these
// builds go beyond kb = 3, to kb = 7 for sectors without poles.
hipError_t qmc_launch_real(int ks, int kb, bool fp32, int variant, bool num,
                           const qmc_launch_args &args, int grid, hipStream_t stream);

// Complex integrand with contour deformation (Eq. 14) for sectors of
// dimension <= dm (dm = qmc_cplx_dm(dim)); polynomial work in FP32 when
// fp32, else FP64; variant 0 built for four waves per SIMD, variant 1 for two.
hipError_t qmc_launch_cplx(int dm, int ks, int kb, bool fp32, int variant,
                           const qmc_launch_args &args, int grid, hipStream_t stream);
int qmc_cplx_dm(int dim);
bool qmc_cplx_supported(int dim, int ks, int kb);

// Fixed-order compensated sum of each group's items.
hipError_t qmc_launch_reduce(const double *partial, const int32_t *viol,
                             const int32_t *group_begin, const int32_t *group_end,
                             int n_groups, int kstride, double *out, int32_t *gviol,
                             hipStream_t stream);

// qmc_math::ln, ln1p, ex, exm1 (fn = 0..3) applied to n device values.
hipError_t qmc_launch_math(int fn, const double *x, double *y, long n, hipStream_t stream);

// Serving: adds each step group's items (fixed order) into the request's
// resident compensated sums dst[g][gks[g]][4]; per-group violation counts.
hipError_t qmc_launch_serve_accumulate(const double *partial, const int32_t *viol,
                                       const int32_t *group_begin, const int32_t *group_end,
                                       double *const *dst, const int32_t *gks, int n_groups,
                                       int kstride, int32_t *gviol, hipStream_t stream);
// Serving: a request's sums [ns][m][kstride][4] combined over sectors per
// shift and order, each sector's series times its coefficient series
// D[ns][QMC_NCOEF][2]: tot[m][n_orders][2].  Order j of tot takes slot
// q = j - e + q_base + ks of a sector with ks poles for D's entry e
// (q_base: lowest order of tot minus the order of D's entry 0).
hipError_t qmc_launch_serve_combine(const double *sums, const qmc_sec_dev *sec, const double *D,
                                    int ns, int m, int kstride, int n_orders, int q_base,
                                    double inv_n, double *tot, hipStream_t stream);
// p[0..n) = v.
hipError_t qmc_launch_fill(double *p, long n, double v, hipStream_t stream);
