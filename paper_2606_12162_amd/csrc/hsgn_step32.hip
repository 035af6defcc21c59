// hsgn_step32.hip -- mixed-precision instantiation of the step kernel (FP32
// storage and arithmetic, FP64 near-shore edges and fix-ups), compiled with
// fused multiply-add contraction.
#include "hsgn_step.hpp"

using namespace hsgn;

void launch_march32(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream)
{
    march_kernel<float, float, true, false><<<nwork, 64, 0, stream>>>(A);
}
