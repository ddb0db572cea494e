// FP64 real integrand kernels for sectors with at most two poles,
// occupancy variant 1 (one wave fewer).
#include "qmc_real.h"

hipError_t qmc_launch_real_lo_v1(int ks, int kb, const qmc_launch_args &args, int grid,
                                 hipStream_t stream)
{
    QMC_REAL_CASES_LO(double, 1, false)
    return hipErrorInvalidValue;
}
