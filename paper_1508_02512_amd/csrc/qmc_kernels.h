// Host-side launchers of the integrand and reduction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_device.h"

// Real (Euclidean) integrand for sectors with `ks` poles carrying ks + kb
// Laurent orders, evaluated in FP64 or FP32; one work-group per item in
// [item_begin, item_end).
hipError_t qmc_launch_real(int ks, int kb, bool fp32, const qmc_launch_args &args, int grid,
                           hipStream_t stream);

// Complex FP64 integrand with contour deformation (Eq. 14) for sectors of
// dimension <= dm (dm = qmc_cplx_dm(dim)).
hipError_t qmc_launch_cplx(int dm, int ks, int kb, const qmc_launch_args &args, int grid,
                           hipStream_t stream);
int qmc_cplx_dm(int dim);
bool qmc_cplx_supported(int dim, int ks, int kb);

// Fixed-order compensated sum of each group's items.
hipError_t qmc_launch_reduce(const double *partial, const int32_t *viol,
                             const int32_t *group_begin, const int32_t *group_end,
                             int n_groups, int kstride, double *out, int32_t *gviol,
                             hipStream_t stream);

// qmc_math::ln, ln1p, ex, exm1 (fn = 0..3) applied to n device values.
hipError_t qmc_launch_math(int fn, const double *x, double *y, long n, hipStream_t stream);
