// FP32-evaluation real integrand kernels (FP64 lattice, shifts and sums),
// occupancy variant 1 (one wave fewer).
#include "qmc_real.h"

hipError_t qmc_launch_real_f32_v1(int ks, int kb, const qmc_launch_args &args, int grid,
                                  hipStream_t stream)
{
    QMC_REAL_CASES_LO(float, 1, false)
    QMC_REAL_CASES_HI(float, 1, false)
    return hipErrorInvalidValue;
}
