// FP64 real integrand kernels for sectors with at most two poles.
#include "qmc_real.h"

hipError_t qmc_launch_real_lo(int ks, int kb, const qmc_launch_args &args, int grid,
                              hipStream_t stream)
{
    QMC_REAL_CASE(0, 1, double) QMC_REAL_CASE(0, 2, double) QMC_REAL_CASE(0, 3, double)
    QMC_REAL_CASE(1, 1, double) QMC_REAL_CASE(1, 2, double) QMC_REAL_CASE(1, 3, double)
    QMC_REAL_CASE(2, 1, double) QMC_REAL_CASE(2, 2, double) QMC_REAL_CASE(2, 3, double)
    return hipErrorInvalidValue;
}
