// Deformed (complex) integrand kernels for sectors of dimension <= 4,
// occupancy variant 1 (two waves).
#include "qmc_cplx.h"

hipError_t qmc_launch_cplx4_v1(int ks, int kb, const qmc_launch_args &args, int grid,
                               hipStream_t stream)
{
    QMC_CPLX_CASE(4, 0, 1, double, 1) QMC_CPLX_CASE(4, 0, 2, double, 1)
    QMC_CPLX_CASE(4, 1, 1, double, 1) QMC_CPLX_CASE(4, 1, 2, double, 1)
    QMC_CPLX_CASE(4, 2, 1, double, 1) QMC_CPLX_CASE(4, 2, 2, double, 1)
    return hipErrorInvalidValue;
}
