// hsgn_step32amr.hip -- mixed-precision step kernel for patches of patch
// sets (stored ghost frames, interface edges, boundary-flux records).
#include "hsgn_step.hpp"

using namespace hsgn;

// blocks of the full kernel over the list of items that need the FP64 edge
// solve when it runs beside the other kernel (beside): one wavefront per
// SIMD of the chip at most, each taking entries in turn
constexpr unsigned FB_BLOCKS_AMR = 1024;

// the full kernel: every item, or with item lists the items that need the
// FP64 edge solve
void launch_march32_amr(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream, bool beside)
{
    const unsigned grid = A.list && beside && nwork > FB_BLOCKS_AMR ? FB_BLOCKS_AMR : nwork;
    if (A.mapped) march_kernel_mapped<float, float, true, true, true><<<grid, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<float, float, true, true, true, true><<<grid, 64, 0, stream>>>(A);
    else march_kernel<float, float, true, true, true, false><<<grid, 64, 0, stream>>>(A);
}

// the kernel without the FP64 edge solve, over the other list
void launch_march32_amr_deep(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream)
{
    const unsigned grid = xcd_grid(nwork);
    if (A.mapped) march_kernel_mapped<float, float, true, false, true><<<grid, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<float, float, true, true, false, true><<<grid, 64, 0, stream>>>(A);
    else march_kernel<float, float, true, true, false, false><<<grid, 64, 0, stream>>>(A);
}

// the item lists from the attempt's input mask, ghost frames included
void launch_classify32_amr(const MarchArgs<float> &A, unsigned nwork, int *cls, hipStream_t stream)
{
    classify_kernel<float, float, true><<<nwork, 64, 0, stream>>>(A, cls);
    list_kernel<LIST_THREADS><<<1, LIST_THREADS, 0, stream>>>(cls, (int)nwork, A.list, A.lcnt,
                                                             A.latch);
}

// the bottom part of the classes, ghost frames included
void launch_static_class32_amr(const MarchArgs<float> &A, unsigned nwork, int *out, hipStream_t stream)
{
    static_class_kernel<float, float, true><<<nwork, 64, 0, stream>>>(A, out);
}
