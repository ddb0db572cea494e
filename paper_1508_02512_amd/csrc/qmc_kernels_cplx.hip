// Dispatch of the deformed (complex) integrand kernels by kernel width.
#include "qmc_kernels.h"

hipError_t qmc_launch_cplx2(int ks, int kb, const qmc_launch_args &args, int grid,
                            hipStream_t stream);
hipError_t qmc_launch_cplx4(int ks, int kb, const qmc_launch_args &args, int grid,
                            hipStream_t stream);
hipError_t qmc_launch_cplx6(int ks, int kb, const qmc_launch_args &args, int grid,
                            hipStream_t stream);
hipError_t qmc_launch_cplx2_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                                hipStream_t stream);
hipError_t qmc_launch_cplx4_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                                hipStream_t stream);
hipError_t qmc_launch_cplx6_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                                hipStream_t stream);

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

hipError_t qmc_launch_cplx(int dm, int ks, int kb, bool fp32, const qmc_launch_args &args,
                           int grid, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (dm == 2) return fp32 ? qmc_launch_cplx2_f32(ks, kb, args, grid, stream)
                             : qmc_launch_cplx2(ks, kb, args, grid, stream);
    if (dm == 4) return fp32 ? qmc_launch_cplx4_f32(ks, kb, args, grid, stream)
                             : qmc_launch_cplx4(ks, kb, args, grid, stream);
    if (dm == 6) return fp32 ? qmc_launch_cplx6_f32(ks, kb, args, grid, stream)
                             : qmc_launch_cplx6(ks, kb, args, grid, stream);
    return hipErrorInvalidValue;
}
