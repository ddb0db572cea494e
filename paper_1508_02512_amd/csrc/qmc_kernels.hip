// Launchers of the real (Euclidean) integrand kernels and the fixed-order
// reduction of per-tile partial sums.
#include <hip/hip_runtime.h>

#include "qmc_common.h"
#include "qmc_device.h"
#include "qmc_kernels.h"
#include "qmc_math.h"

using namespace qmc;

hipError_t qmc_launch_real_lo(int ks, int kb, const qmc_launch_args &args, int grid,
                              hipStream_t stream);
hipError_t qmc_launch_real_hi(int ks, int kb, const qmc_launch_args &args, int grid,
                              hipStream_t stream);
hipError_t qmc_launch_real_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                               hipStream_t stream);

hipError_t qmc_launch_real(int ks, int kb, bool fp32, const qmc_launch_args &args, int grid,
                           hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (fp32) return qmc_launch_real_f32(ks, kb, args, grid, stream);
    return ks <= 2 ? qmc_launch_real_lo(ks, kb, args, grid, stream)
                   : qmc_launch_real_hi(ks, kb, args, grid, stream);
}

// Fixed-order compensated sum of the tiles of every output group.
__global__ void qmc_reduce_groups(const double *partial, const int32_t *viol,
                                  const int32_t *group_begin, const int32_t *group_end,
                                  int n_groups, int kstride, double *out, int32_t *gviol)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = (int)(tid / kstride), q = (int)(tid % kstride);
    if (g >= n_groups) return;
    const int i0 = group_begin[g], i1 = group_end[g];
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    int v = 0;
    for (int i = i0; i < i1; ++i) {
        const double *p = partial + ((size_t)i * kstride + q) * 4;
        double e;
        two_sum(sr, p[0], sr, e);
        cr += p[1] + e;
        two_sum(si, p[2], si, e);
        ci += p[3] + e;
        if (q == 0) v += viol[i];
    }
    out[((size_t)g * kstride + q) * 2] = sr + cr;
    out[((size_t)g * kstride + q) * 2 + 1] = si + ci;
    if (q == 0) gviol[g] = v;
}

hipError_t qmc_launch_reduce(const double *partial, const int32_t *viol,
                             const int32_t *group_begin, const int32_t *group_end,
                             int n_groups, int kstride, double *out, int32_t *gviol,
                             hipStream_t stream)
{
    const long total = (long)n_groups * kstride;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (int)((total + threads - 1) / threads);
    hipLaunchKernelGGL(qmc_reduce_groups, dim3(blocks), dim3(threads), 0, stream,
                       partial, viol, group_begin, group_end, n_groups, kstride, out,
                       gviol);
    return hipGetLastError();
}

// Elementary functions of the integrand kernels on an array (diagnostics).
__global__ void qmc_math_kernel(int fn, const double *x, double *y, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    double r = 0.0;
    switch (fn) {
    case 0: r = qmc_math::ln(v); break;
    case 1: r = qmc_math::ln1p(v); break;
    case 2: r = qmc_math::ex(v); break;
    default: r = qmc_math::exm1(v); break;
    }
    y[i] = r;
}

hipError_t qmc_launch_math(int fn, const double *x, double *y, long n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const long blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(qmc_math_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, fn,
                       x, y, n);
    return hipGetLastError();
}
