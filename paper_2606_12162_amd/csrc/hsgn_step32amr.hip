// hsgn_step32amr.hip -- mixed-precision step kernel for patches of patch
// sets (stored ghost frames, interface edges, boundary-flux records).
#include "hsgn_step.hpp"

using namespace hsgn;

void launch_march32_amr(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream)
{
    march_kernel<float, float, true, true><<<nwork, 64, 0, stream>>>(A);
}
