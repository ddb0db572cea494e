// Dispatch of the deformed (complex) integrand kernels by kernel width.
#include "qmc_kernels.h"

#define QMC_CPLX_LAUNCHER(name)                                                      \
    hipError_t name(int ks, int kb, const qmc_launch_args &args, int grid, hipStream_t stream);
QMC_CPLX_LAUNCHER(qmc_launch_cplx2)
QMC_CPLX_LAUNCHER(qmc_launch_cplx4)
QMC_CPLX_LAUNCHER(qmc_launch_cplx6)
QMC_CPLX_LAUNCHER(qmc_launch_cplx2_f32)
QMC_CPLX_LAUNCHER(qmc_launch_cplx4_f32)
QMC_CPLX_LAUNCHER(qmc_launch_cplx6_f32)
QMC_CPLX_LAUNCHER(qmc_launch_cplx2_v1)
QMC_CPLX_LAUNCHER(qmc_launch_cplx4_v1)
QMC_CPLX_LAUNCHER(qmc_launch_cplx6_v1)
QMC_CPLX_LAUNCHER(qmc_launch_cplx2_f32_v1)
QMC_CPLX_LAUNCHER(qmc_launch_cplx4_f32_v1)
QMC_CPLX_LAUNCHER(qmc_launch_cplx6_f32_v1)

int qmc_cplx_dm(int dim) { return dim <= 2 ? 2 : dim <= 4 ? 4 : dim <= 6 ? 6 : 0; }

// Deformed sectors: dimension <= 6, at most two poles, one or two orders
// above the poles (three for dimension <= 2).  The deformed kernel forms
// the mixed differences of Eq. 11 from corner values; with three or four
// poles that loses up to ~1e-10 and ~5e-9 of the summed magnitudes to
// cancellation, short of FP64 accuracy, so such sectors are refused.
bool qmc_cplx_supported(int dim, int ks, int kb)
{
    const int dm = qmc_cplx_dm(dim);
    return dm != 0 && ks >= 0 && ks <= 2 && kb >= 1 && kb <= (dm == 2 ? 3 : 2);
}

hipError_t qmc_launch_cplx(int dm, int ks, int kb, bool fp32, int variant,
                           const qmc_launch_args &args, int grid, hipStream_t stream)
{
    typedef hipError_t (*launcher)(int, int, const qmc_launch_args &, int, hipStream_t);
    // [variant][fp32][width 2, 4, 6]
    static const launcher table[2][2][3] = {
        {{qmc_launch_cplx2, qmc_launch_cplx4, qmc_launch_cplx6},
         {qmc_launch_cplx2_f32, qmc_launch_cplx4_f32, qmc_launch_cplx6_f32}},
        {{qmc_launch_cplx2_v1, qmc_launch_cplx4_v1, qmc_launch_cplx6_v1},
         {qmc_launch_cplx2_f32_v1, qmc_launch_cplx4_f32_v1, qmc_launch_cplx6_f32_v1}}};
    if (grid <= 0) return hipSuccess;
    if (variant < 0 || variant > 1 || (dm != 2 && dm != 4 && dm != 6)) return hipErrorInvalidValue;
    return table[variant][fp32 ? 1 : 0][dm / 2 - 1](ks, kb, args, grid, stream);
}
