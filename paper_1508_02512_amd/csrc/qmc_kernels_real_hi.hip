// FP64 real integrand kernels for sectors with three or four poles.
#include "qmc_real.h"

hipError_t qmc_launch_real_hi(int ks, int kb, const qmc_launch_args &args, int grid,
                              hipStream_t stream)
{
    QMC_REAL_CASE(3, 1, double) QMC_REAL_CASE(3, 2, double) QMC_REAL_CASE(3, 3, double)
    QMC_REAL_CASE(4, 1, double) QMC_REAL_CASE(4, 2, double) QMC_REAL_CASE(4, 3, double)
    return hipErrorInvalidValue;
}
