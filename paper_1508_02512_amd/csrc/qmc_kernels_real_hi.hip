// FP64 real integrand kernels for sectors with three or four poles.
#include "qmc_real.h"

hipError_t qmc_launch_real_hi(int ks, int kb, const qmc_launch_args &args, int grid,
                              hipStream_t stream)
{
    QMC_REAL_CASES_HI(double, 0, false)
    return hipErrorInvalidValue;
}
