// FP64 real integrand kernels with numerator factors for pole-free sectors
// carrying 4-7 orders: the sectors that integration by parts (Eq. 13)
// leaves when it is taken at the poles as well.
#include "qmc_real.h"

hipError_t qmc_launch_real_num_wide(int ks, int kb, const qmc_launch_args &args, int grid,
                                    hipStream_t stream)
{
    QMC_REAL_CASES_WIDE(double, 0, true)
    return hipErrorInvalidValue;
}
