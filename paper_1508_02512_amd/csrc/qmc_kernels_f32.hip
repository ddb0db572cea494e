// FP32-evaluation real integrand kernels (FP64 lattice, shifts and sums).
#include "qmc_real.h"

hipError_t qmc_launch_real_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                               hipStream_t stream)
{
    QMC_REAL_CASES_LO(float, 0, false)
    QMC_REAL_CASES_HI(float, 0, false)
    return hipErrorInvalidValue;
}
