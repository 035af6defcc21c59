// hsgn_step64amr.hip -- FP64 step kernel for patches of patch sets (stored
// ghost frames, interface edges, boundary-flux records).
#include "hsgn_step.hpp"

using namespace hsgn;

void launch_march64_amr(const MarchArgs<double> &A, unsigned nwork, hipStream_t stream)
{
    const unsigned grid = xcd_grid(nwork);
    if (A.mapped) march_kernel_mapped<double, double, false, true, true><<<grid, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<double, double, false, true, true, true><<<grid, 64, 0, stream>>>(A);
    else march_kernel<double, double, false, true, true, false><<<grid, 64, 0, stream>>>(A);
}
