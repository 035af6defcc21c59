// hsgn_step64.hip -- FP64 instantiation of the step kernel (its own
// translation unit, so that the FP64 and FP32 instances compile in parallel).
#include "hsgn_step.hpp"

using namespace hsgn;

void launch_march64(const MarchArgs<double> &A, unsigned nwork, hipStream_t stream)
{
    const unsigned grid = xcd_grid(nwork);
    if (A.mapped) march_kernel_mapped<double, double, false><<<grid, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<double, double, false, false, true, true><<<grid, 64, 0, stream>>>(A);
    else march_kernel<double, double, false, false, true, false><<<grid, 64, 0, stream>>>(A);
}
