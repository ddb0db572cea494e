// Deformed integrand kernels, FP32 evaluation mode, for sectors of dimension <= 6.
#include "qmc_cplx.h"

hipError_t qmc_launch_cplx6_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                                 hipStream_t stream)
{
    QMC_CPLX_CASE(6, 0, 1, float, 0) QMC_CPLX_CASE(6, 0, 2, float, 0)
    QMC_CPLX_CASE(6, 1, 1, float, 0) QMC_CPLX_CASE(6, 1, 2, float, 0)
    QMC_CPLX_CASE(6, 2, 1, float, 0) QMC_CPLX_CASE(6, 2, 2, float, 0)
    return hipErrorInvalidValue;
}
