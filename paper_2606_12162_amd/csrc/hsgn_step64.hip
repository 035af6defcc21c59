// hsgn_step64.hip -- FP64 instantiation of the step kernel (its own
// translation unit, so that the FP64 and FP32 instances compile in parallel).
#include "hsgn_step.hpp"

using namespace hsgn;

void launch_march64(const MarchArgs<double> &A, unsigned nwork, hipStream_t stream)
{
    if (A.mapped) march_kernel_mapped<double, double, false><<<nwork, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<double, double, false, false, true, true><<<nwork, 64, 0, stream>>>(A);
    else march_kernel<double, double, false, false, true, false><<<nwork, 64, 0, stream>>>(A);
}
