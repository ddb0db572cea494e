// Launchers of the real (Euclidean) integrand kernels and the fixed-order
// reduction of per-tile partial sums.
#include <hip/hip_runtime.h>

#include "qmc_common.h"
#include "qmc_device.h"
#include "qmc_kernels.h"
#include "qmc_math.h"

using namespace qmc;

#define QMC_REAL_LAUNCHER(name)                                                      \
    hipError_t name(int ks, int kb, const qmc_launch_args &args, int grid, hipStream_t stream);
QMC_REAL_LAUNCHER(qmc_launch_real_lo)
QMC_REAL_LAUNCHER(qmc_launch_real_hi)
QMC_REAL_LAUNCHER(qmc_launch_real_f32)
QMC_REAL_LAUNCHER(qmc_launch_real_lo_v1)
QMC_REAL_LAUNCHER(qmc_launch_real_hi_v1)
QMC_REAL_LAUNCHER(qmc_launch_real_f32_v1)
QMC_REAL_LAUNCHER(qmc_launch_real_num_lo)
QMC_REAL_LAUNCHER(qmc_launch_real_num_hi)
QMC_REAL_LAUNCHER(qmc_launch_real_num_f32)
QMC_REAL_LAUNCHER(qmc_launch_real_num_wide)

hipError_t qmc_launch_real(int ks, int kb, bool fp32, int variant, bool num,
                           const qmc_launch_args &args, int grid, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (num) {   // one occupancy build: these classes are small
        if (fp32) return qmc_launch_real_num_f32(ks, kb, args, grid, stream);
        if (kb > 3) return qmc_launch_real_num_wide(ks, kb, args, grid, stream);
        return ks <= 2 ? qmc_launch_real_num_lo(ks, kb, args, grid, stream)
                       : qmc_launch_real_num_hi(ks, kb, args, grid, stream);
    }
    if (variant == 1) {
        if (fp32) return qmc_launch_real_f32_v1(ks, kb, args, grid, stream);
        return ks <= 2 ? qmc_launch_real_lo_v1(ks, kb, args, grid, stream)
                       : qmc_launch_real_hi_v1(ks, kb, args, grid, stream);
    }
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
    const float vf = (float)v;
    double r = 0.0;
    switch (fn) {
    case 0: r = qmc_math::ln(v); break;
    case 1: r = qmc_math::ln1p(v); break;
    case 2: r = qmc_math::ex(v); break;
    case 3: r = qmc_math::exm1(v); break;
    case 4: r = qmc_math::rcp(v); break;
    // the float overloads of FP32 evaluation, on x rounded to float
    case 5: r = qmc_math::ln(vf); break;
    case 6: r = qmc_math::ln1p(vf); break;
    case 7: r = qmc_math::ex(vf); break;
    default: r = qmc_math::exm1(vf); break;
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

// Serving: the items of each group of one step added, one at a time in item
// order, into the request's resident compensated sums (TwoSum):
// dst[g][q] = (re hi, re lo, im hi, im lo) of order slot q < gks[g] (the
// group's own slots; the step's partial slots may be wider).  Adding item by
// item makes the sums independent of how a level's items are cut into steps.
__global__ void qmc_serve_accumulate_k(const double *partial, const int32_t *viol,
                                       const int32_t *group_begin, const int32_t *group_end,
                                       double *const *dst, const int32_t *gks, int n_groups,
                                       int kstride, int32_t *gviol)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = (int)(tid / kstride), q = (int)(tid % kstride);
    if (g >= n_groups || q >= gks[g]) return;
    const int i0 = group_begin[g], i1 = group_end[g];
    double *d = dst[g] + (size_t)q * 4;
    double hr = d[0], lr = d[1], hi = d[2], li = d[3];
    int v = 0;
    for (int i = i0; i < i1; ++i) {
        const double *p = partial + ((size_t)i * kstride + q) * 4;
        double e;
        two_sum(hr, p[0], hr, e);
        lr += e + p[1];
        two_sum(hi, p[2], hi, e);
        li += e + p[3];
        if (q == 0) v += viol[i];
    }
    d[0] = hr;
    d[1] = lr;
    d[2] = hi;
    d[3] = li;
    if (q == 0) gviol[g] = v;
}

hipError_t qmc_launch_serve_accumulate(const double *partial, const int32_t *viol,
                                       const int32_t *group_begin, const int32_t *group_end,
                                       double *const *dst, const int32_t *gks, int n_groups,
                                       int kstride, int32_t *gviol, hipStream_t stream)
{
    const long total = (long)n_groups * kstride;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(qmc_serve_accumulate_k, dim3((unsigned)((total + threads - 1) / threads)),
                       dim3(threads), 0, stream, partial, viol, group_begin, group_end, dst,
                       gks, n_groups, kstride, gviol);
    return hipGetLastError();
}

// Serving: one request's resident sums combined over sectors for every
// shift k and sector Laurent order j (Eq. 19 before the prefactor):
//   tot[k][j] = sum_s D_s (hi + lo)_{s,k,q} / n,  q = j + sec_lo + ks_s,
// each sum compensated, sectors in index order.  One thread per (k, j).
__global__ void qmc_serve_combine_k(const double *sums, const qmc_sec_dev *sec,
                                    const double *D, int ns, int m, int kstride, int n_orders,
                                    int q_base, double inv_n, double *tot)
{
    const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (tid >= m * n_orders) return;
    const int k = tid / n_orders, j = tid % n_orders;
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int s = 0; s < ns; ++s) {
        // order j of the sum times C(eps): sum_e C_e v_{j-e}, with the
        // orders of the total, of C and of the sector's slots offset by q_base
        for (int e = 0; e < QMC_NCOEF; ++e) {
            const double dr = D[2 * (s * QMC_NCOEF + e)];
            const double di = D[2 * (s * QMC_NCOEF + e) + 1];
            if (dr == 0.0 && di == 0.0) continue;
            const int q = j - e + q_base + sec[s].ks;
            if (q < 0 || q >= sec[s].K) continue;
            const double *p = sums + (((size_t)s * m + k) * kstride + q) * 4;
            const double vr = (p[0] + p[1]) * inv_n, vi = (p[2] + p[3]) * inv_n;
            double x;
            two_sum(sr, dr * vr - di * vi, sr, x);
            cr += x;
            two_sum(si, dr * vi + di * vr, si, x);
            ci += x;
        }
    }
    tot[2 * tid] = sr + cr;
    tot[2 * tid + 1] = si + ci;
}

hipError_t qmc_launch_serve_combine(const double *sums, const qmc_sec_dev *sec, const double *D,
                                    int ns, int m, int kstride, int n_orders, int q_base,
                                    double inv_n, double *tot, hipStream_t stream)
{
    const int total = m * n_orders;
    if (total == 0) return hipSuccess;
    const int threads = 64;
    hipLaunchKernelGGL(qmc_serve_combine_k, dim3((total + threads - 1) / threads),
                       dim3(threads), 0, stream, sums, sec, D, ns, m, kstride, n_orders,
                       q_base, inv_n, tot);
    return hipGetLastError();
}

// Fills n doubles with v (graph-safe clearing; no memset node).
__global__ void qmc_fill_k(double *p, long n, double v)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t qmc_launch_fill(double *p, long n, double v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(qmc_fill_k, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads),
                       0, stream, p, n, v);
    return hipGetLastError();
}
