// Deformed (complex) integrand kernels for sectors of dimension <= 6,
// occupancy variant 1 (two waves).
#include "qmc_cplx.h"

hipError_t qmc_launch_cplx6_v1(int ks, int kb, const qmc_launch_args &args, int grid,
                               hipStream_t stream)
{
    QMC_CPLX_CASE(6, 0, 1, double, 1) QMC_CPLX_CASE(6, 0, 2, double, 1)
    QMC_CPLX_CASE(6, 1, 1, double, 1) QMC_CPLX_CASE(6, 1, 2, double, 1)
    QMC_CPLX_CASE(6, 2, 1, double, 1) QMC_CPLX_CASE(6, 2, 2, double, 1)
    return hipErrorInvalidValue;
}
