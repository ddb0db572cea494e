// Deformed (complex) integrand kernels for sectors of dimension <= 2,
// occupancy variant 1 (two waves).
#include "qmc_cplx.h"

hipError_t qmc_launch_cplx2_v1(int ks, int kb, const qmc_launch_args &args, int grid,
                               hipStream_t stream)
{
    QMC_CPLX_CASE(2, 0, 1, double, 1) QMC_CPLX_CASE(2, 0, 2, double, 1)
    QMC_CPLX_CASE(2, 1, 1, double, 1) QMC_CPLX_CASE(2, 1, 2, double, 1)
    QMC_CPLX_CASE(2, 2, 1, double, 1) QMC_CPLX_CASE(2, 2, 2, double, 1)
    QMC_CPLX_CASE(2, 0, 3, double, 1) QMC_CPLX_CASE(2, 1, 3, double, 1) QMC_CPLX_CASE(2, 2, 3, double, 1)
    return hipErrorInvalidValue;
}
