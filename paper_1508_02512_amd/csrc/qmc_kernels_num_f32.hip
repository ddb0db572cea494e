// FP32-evaluation real integrand kernels with numerator factors
// (integration by parts, Eq. 13).
#include "qmc_real.h"

hipError_t qmc_launch_real_num_f32(int ks, int kb, const qmc_launch_args &args, int grid,
                                   hipStream_t stream)
{
    QMC_REAL_CASES_LO(float, 0, true)
    QMC_REAL_CASES_HI(float, 0, true)
    QMC_REAL_CASES_WIDE(float, 0, true)
    return hipErrorInvalidValue;
}
