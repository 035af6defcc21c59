#pragma once
// hsgn_step.hpp -- the marching step kernel and its wavefront lane policy.

#include <hip/hip_runtime.h>

#include "hsgn_march.hpp"

namespace hsgn {

// whole-wavefront lane shifts through DPP (GFX9 wave_shr:1 / wave_shl:1):
// lane i receives lane i-1 (up) or lane i+1 (down) as a VALU operand
// modifier, without a trip through the LDS crossbar.  Lane 0 (up) and lane
// 63 (down) keep their own value; they are halo lanes whose results are
// never used.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

__device__ inline int dpp_up(int x) { return __builtin_amdgcn_update_dpp(x, x, DPP_WAVE_SHR1, 0xf, 0xf, false); }
__device__ inline int dpp_dn(int x) { return __builtin_amdgcn_update_dpp(x, x, DPP_WAVE_SHL1, 0xf, 0xf, false); }

template <class T>
struct GpuLanes {
    T *ring_;
    __device__ T *ring() const { return ring_; }
    __device__ int lane() const { return (int)(threadIdx.x & 63); }
    __device__ float up(float x) const { return __int_as_float(dpp_up(__float_as_int(x))); }
    __device__ float dn(float x) const { return __int_as_float(dpp_dn(__float_as_int(x))); }
    __device__ double up(double x) const
    {
        long long v = __double_as_longlong(x);
        int lo = dpp_up((int)(v & 0xffffffffLL)), hi = dpp_up((int)(v >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    __device__ double dn(double x) const
    {
        long long v = __double_as_longlong(x);
        int lo = dpp_dn((int)(v & 0xffffffffLL)), hi = dpp_dn((int)(v >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    __device__ int upi(int x) const { return dpp_up(x); }
    __device__ int dni(int x) const { return dpp_dn(x); }
    __device__ bool any(int p) const { return __any(p); }
    template <class S>
    __device__ void finish(const MarchArgs<S> &A, int wid, int scen, double rx, double ry,
                           double clip) const
    {
        for (int o = 32; o > 0; o >>= 1) {
            rx = fmax(rx, __shfl_xor(rx, o, 64));
            ry = fmax(ry, __shfl_xor(ry, o, 64));
            clip += __shfl_xor(clip, o, 64);
        }
        if (lane() == 0) {
            atomicMax(&A.scen[scen].rx_bits, (unsigned long long)__double_as_longlong(rx));
            atomicMax(&A.scen[scen].ry_bits, (unsigned long long)__double_as_longlong(ry));
            A.clip_slots[wid] = clip;
        }
    }
};

// Mixed precision runs two wavefronts per SIMD: registers are capped at
// 256 per lane (the few values beyond that spill to scratch), which hides
// more latency than the spills cost.  FP64 keeps one wavefront per SIMD
// with its values in VGPRs and AGPRs.
//
// With item lists (A.list) the kernel takes the items of its class's list:
// FB false the items none of whose edges takes the FP64 solve, compiled
// without it (its registers then fit without spilling), one block per
// entry; FB true the others, on fewer blocks than the work table has items,
// each block taking entries b, b + grid, ... in turn.
template <class S, class T, bool MIXED, bool AMR, bool FB = true>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MIXED ? 2 : 1, MIXED ? 2 : 1)))
void march_kernel(MarchArgs<S> A)
{
    __shared__ T ring[3 * EIG_FIELDS * 64 + (MIXED ? 3 * 7 * 64 : 0)];
    GpuLanes<T> ln{ring};
    if (MIXED && !AMR && FB) {
        const unsigned n = A.list ? A.lcnt[1] : (unsigned)A.nwork;
        for (unsigned b = blockIdx.x; b < n; b += gridDim.x) {     // uniform over the wavefront
            const int wid = A.list ? A.list[A.nwork + (int)b] : (int)b;
            march<GpuLanes<T>, S, T, MIXED, AMR, FB>(ln, A, wid);
        }
    } else {
        int wid = (int)blockIdx.x;
        if (wid >= A.nwork) return;
        if (A.list) {                                               // uniform over the wavefront
            if ((unsigned)wid >= A.lcnt[0]) return;
            wid = A.list[wid];
        }
        march<GpuLanes<T>, S, T, MIXED, AMR, FB>(ln, A, wid);
    }
}

// The cells a single-grid work item's wavefront loads: columns i0-2..i0+61
// clamped as the step clamps them, rows r0-2..r0+th+1, through the boundary
// map.  A cell has c^2 = 0 when its mask puts it in the SWE region or
// breaking, or when its bottom alone gives c^2 = 0 (relax_c2 with phi_T = 1
// is then zero); the two parts are tested apart.

// the bottom part, per item, recomputed when the bathymetry or the work
// table changes
template <class S, class T>
__global__ __launch_bounds__(64) void static_class_kernel(MarchArgs<S> A, int *out)
{
    int wid = (int)blockIdx.x;
    if (wid >= A.nwork) return;
    const WorkItem wk = A.work[wid];
    const PatchInfo pi = A.patches[wk.patch];
    const int lane = (int)(threadIdx.x & 63);
    int col = wk.i0 - 2 + lane;
    if (col > pi.nx + 1) col = pi.nx + 1;
    int fx = 0, fy = 0;
    const int mc = map_index(col, pi.nx, pi.bc[0], pi.bc[1], &fx);
    int hot = 0;
    for (int k = wk.r0 - 2; k <= wk.r0 + wk.th + 1; k++) {
        const int mr = map_index(k, pi.ny, pi.bc[2], pi.bc[3], &fy);
        const long long idx = pi.coff + (long long)mr * pi.pitch + mc;
        hot |= !(relax_c2(A.P, MASK_PHI, (T)A.bath[idx]) > (T)0);
    }
    const int any_hot = __any(hot);
    if (lane == 0) out[wid] = any_hot ? 1 : 0;
}

// class of each item for the coming attempt from the attempt's input mask
// and the bottom part, into cls[wid] (0: no cell the item loads has c^2 =
// 0, so that none of its edges needs the FP64 solve; 1: the others).  One
// wavefront per item.
template <class S, class T>
__global__ __launch_bounds__(64) void classify_kernel(MarchArgs<S> A, int *cls)
{
    int wid = (int)blockIdx.x;
    if (wid >= A.nwork) return;
    const int lane = (int)(threadIdx.x & 63);
    if (A.clsb[wid]) {                          // uniform over the wavefront
        if (lane == 0) cls[wid] = 1;
        return;
    }
    const WorkItem wk = A.work[wid];
    const PatchInfo pi = A.patches[wk.patch];
    const uint8_t *mk = A.scen[pi.scen].cur ? A.m1 : A.m0;
    int col = wk.i0 - 2 + lane;
    if (col > pi.nx + 1) col = pi.nx + 1;
    int fx = 0, fy = 0;
    const int mc = map_index(col, pi.nx, pi.bc[0], pi.bc[1], &fx);
    int hot = 0;
#pragma unroll 8
    for (int k = wk.r0 - 2; k <= wk.r0 + wk.th + 1; k++) {
        const int mr = map_index(k, pi.ny, pi.bc[2], pi.bc[3], &fy);
        const int m = mk[pi.coff + (long long)mr * pi.pitch + mc];
        hot |= (m & (MASK_PHI | MASK_BRK)) != MASK_PHI;
    }
    const int any_hot = __any(hot);
    if (lane == 0) cls[wid] = any_hot ? 1 : 0;
}

// the two item lists from the classes, each in ascending item order, and
// their lengths: one workgroup of LIST_THREADS threads, thread t scanning a
// contiguous run of the classes
constexpr int LIST_THREADS = 1024;

template <int NT>
__global__ __launch_bounds__(NT) void list_kernel(const int *cls, int nwork, int *list,
                                                            unsigned *lcnt)
{
    __shared__ int part[2][NT];
    const int t = (int)threadIdx.x;
    const int per = (nwork + NT - 1) / NT;
    const int a = t * per < nwork ? t * per : nwork;
    const int e = a + per < nwork ? a + per : nwork;
    int n1 = 0;
    for (int w = a; w < e; w++) n1 += cls[w];
    part[0][t] = (e - a) - n1;
    part[1][t] = n1;
    __syncthreads();
    // inclusive scans of both counts (Hillis-Steele over the workgroup)
    for (int o = 1; o < NT; o <<= 1) {
        int x0 = t >= o ? part[0][t - o] : 0, x1 = t >= o ? part[1][t - o] : 0;
        __syncthreads();
        part[0][t] += x0;
        part[1][t] += x1;
        __syncthreads();
    }
    int p0 = part[0][t] - ((e - a) - n1), p1 = part[1][t] - n1;
    for (int w = a; w < e; w++) {
        if (cls[w]) list[nwork + p1++] = w;
        else list[p0++] = w;
    }
    if (t == NT - 1) {
        lcnt[0] = (unsigned)part[0][t];
        lcnt[1] = (unsigned)part[1][t];
    }
}


}  // namespace hsgn
