// hsgn_step32.hip -- mixed-precision instantiation of the step kernel (FP32
// storage and arithmetic, FP64 near-shore edges and fix-ups), compiled with
// fused multiply-add contraction.
#include "hsgn_step.hpp"

using namespace hsgn;

// blocks of the full kernel over the list of items that need the FP64 edge
// solve when it runs beside the other kernel (beside): one wavefront per
// SIMD of the chip at most, each taking entries in turn, so that the list's
// items start at once
constexpr unsigned FB_BLOCKS = 1024;

// the full kernel: every item, or with item lists the items that need the
// FP64 edge solve
void launch_march32(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream, bool beside)
{
    const unsigned grid = A.list && beside && nwork > FB_BLOCKS ? FB_BLOCKS : nwork;
    if (A.mapped) march_kernel_mapped<float, float, true, true><<<grid, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<float, float, true, false, true, true><<<grid, 64, 0, stream>>>(A);
    else march_kernel<float, float, true, false, true, false><<<grid, 64, 0, stream>>>(A);
}

// the kernel without the FP64 edge solve, over the other list
void launch_march32_deep(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream)
{
    const unsigned grid = xcd_grid(nwork);
    if (A.mapped) march_kernel_mapped<float, float, true, false><<<grid, 64, 0, stream>>>(A);
    else if (A.sponge) march_kernel<float, float, true, false, false, true><<<grid, 64, 0, stream>>>(A);
    else march_kernel<float, float, true, false, false, false><<<grid, 64, 0, stream>>>(A);
}

// the item lists from the attempt's input mask (classes into cls)
void launch_classify32(const MarchArgs<float> &A, unsigned nwork, int *cls, hipStream_t stream)
{
    classify_kernel<float, float, false><<<nwork, 64, 0, stream>>>(A, cls);
    list_kernel<LIST_THREADS><<<1, LIST_THREADS, 0, stream>>>(cls, (int)nwork, A.list, A.lcnt,
                                                             A.latch);
}

// the bottom part of the classes (after a bathymetry or work-table change)
void launch_static_class32(const MarchArgs<float> &A, unsigned nwork, int *out, hipStream_t stream)
{
    static_class_kernel<float, float, false><<<nwork, 64, 0, stream>>>(A, out);
}
