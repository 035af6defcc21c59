#pragma once
// hsgn_step.hpp -- the marching step kernel and its wavefront lane policy.

#include <hip/hip_runtime.h>

#include "hsgn_march.hpp"

namespace hsgn {

// whole-wavefront lane shifts through DPP (GFX9 wave_shr:1 / wave_shl:1):
// lane i receives lane i-1 (up) or lane i+1 (down) as a VALU operand
// modifier, without a trip through the LDS crossbar.  Lane 0 (up) and lane
// 63 (down) have no source and receive zero (bound control), so a shift is
// one instruction with no copy of the old value; they are halo lanes whose
// results are never stored and are left out of the Courant maxima, the
// clipped mass and the error flags.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

__device__ inline int dpp_up(int x) { return __builtin_amdgcn_update_dpp(0, x, DPP_WAVE_SHR1, 0xf, 0xf, true); }
__device__ inline int dpp_dn(int x) { return __builtin_amdgcn_update_dpp(0, x, DPP_WAVE_SHL1, 0xf, 0xf, true); }

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

// XCD-aware order: the chip hands consecutive blocks of a launch to its 8
// XCDs in turn, and each XCD has its own L2.  Block b takes item
// (b mod 8) per + b / 8 (per = ceil(n / 8)), so that each XCD works through
// one contiguous run of the work table (row-tile major), where neighbouring
// strips, which share halo columns and cache lines, meet in the same L2.
// Launches over one block per item cover n rounded up to a multiple of 8
// (xcd_grid).  False: the block has no item.
constexpr unsigned XCDS = 8;
__device__ inline bool xcd_item(unsigned b, unsigned n, int &item)
{
    const unsigned per = (n + XCDS - 1) / XCDS, j = b / XCDS;
    item = (int)((b % XCDS) * per + j);
    return j < per && (unsigned)item < n;
}
inline unsigned xcd_grid(unsigned n) { return (n + XCDS - 1) / XCDS * XCDS; }

// Occupancy: the mixed-precision kernel without the FP64 edge solve (FB
// false) fits in about 200 registers and runs two wavefronts per SIMD.  The
// kernels with it (mixed FB true, which takes only the coastal items beside
// the other, and FP64) run one wavefront per SIMD with their values in VGPRs
// and AGPRs: capped at 256 registers for two, the mixed full kernel spilled
// 152 bytes per lane to scratch and held its CUs longer than the wait it
// hid.
//
// With item lists (A.list) the kernel takes the items of its class's list:
// FB false the items none of whose edges takes the FP64 solve, compiled
// without it (its registers then fit without spilling), one block per
// entry; FB true the others, block b taking entries b, b + grid, ... in turn
// (launched on fewer blocks than the work table has items when it runs
// beside the other kernel).
//
// SP: compiled with the sponge relaxation (launched when some patch has a
// sponge; the kernels without it keep their registers).
template <class S, class T, bool MIXED, bool AMR, bool FB = true, bool SP = false>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu((MIXED && !FB) ? 2 : 1, (MIXED && !FB) ? 2 : 1)))
void march_kernel(MarchArgs<S> A)
{
    __shared__ T ring[3 * EIG_FIELDS * 64 + (MIXED ? 3 * 7 * 64 : (PARK_WAVES + PARK_SIDE) * 64)];
    GpuLanes<T> ln{ring};
    if (MIXED && FB) {
        const unsigned n = A.list ? A.lcnt[1] : (unsigned)A.nwork;
        for (unsigned b = blockIdx.x; b < n; b += gridDim.x) {     // uniform over the wavefront
            const int wid = A.list ? A.list[A.nwork + (int)b] : (int)b;
            march<GpuLanes<T>, S, T, MIXED, AMR, FB, SP>(ln, A, wid);
        }
    } else {
        const unsigned n = A.list ? A.lcnt[0] : (unsigned)A.nwork;
        int wid;
        if (!xcd_item(blockIdx.x, n, wid)) return;                 // uniform over the wavefront
        if (A.list) wid = A.list[wid];
        march<GpuLanes<T>, S, T, MIXED, AMR, FB, SP>(ln, A, wid);
    }
}

// the step on mapped grids (launched for the whole work table when some
// patch is mapped; AMR: the patches of patch sets), with the x-edge frames
// also kept in the LDS ring; items and lists as in march_kernel
template <class S, class T, bool MIXED, bool FB = true, bool AMR = false>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu((MIXED && !FB) ? 2 : 1, (MIXED && !FB) ? 2 : 1)))
void march_kernel_mapped(MarchArgs<S> A)
{
    __shared__ T ring[3 * (EIG_FIELDS + 5) * 64 + (MIXED ? 3 * 7 * 64 : 0)];
    GpuLanes<T> ln{ring};
    if (MIXED && FB) {
        const unsigned n = A.list ? A.lcnt[1] : (unsigned)A.nwork;
        for (unsigned b = blockIdx.x; b < n; b += gridDim.x) {     // uniform over the wavefront
            const int wid = A.list ? A.list[A.nwork + (int)b] : (int)b;
            march<GpuLanes<T>, S, T, MIXED, AMR, FB, false, true>(ln, A, wid);
        }
    } else {
        const unsigned n = A.list ? A.lcnt[0] : (unsigned)A.nwork;
        int wid;
        if (!xcd_item(blockIdx.x, n, wid)) return;                 // uniform over the wavefront
        if (A.list) wid = A.list[wid];
        march<GpuLanes<T>, S, T, MIXED, AMR, FB, false, true>(ln, A, wid);
    }
}

// The cells a work item's wavefront loads: columns i0-2..i0+61 clamped as
// the step clamps them, rows r0-2..r0+th+1, through the boundary map (single
// grids) or from the stored ghost frame (FRAMED, patches of patch sets).  A cell has c^2 = 0 when its mask puts it in the SWE region or
// breaking, or when its bottom alone gives c^2 = 0 (relax_c2 with phi_T = 1
// is then zero); the two parts are tested apart.

// the bottom part, per item, recomputed when the bathymetry or the work
// table changes
template <bool FRAMED>
HSGN_HD int footprint_col(const PatchInfo &pi, int i0, int lane)
{
    int col = i0 - 2 + lane;
    if (col > pi.nx + 1) col = pi.nx + 1;
    int fx = 0;
    return FRAMED ? col : map_index(col, pi.nx, pi.bc[0], pi.bc[1], &fx);
}

template <bool FRAMED>
HSGN_HD long long footprint_row(const PatchInfo &pi, int k)
{
    int fy = 0;
    const int mr = FRAMED ? k : map_index(k, pi.ny, pi.bc[2], pi.bc[3], &fy);
    return pi.coff + (long long)mr * pi.pitch;
}

template <class S, class T, bool FRAMED>
__global__ __launch_bounds__(64) void static_class_kernel(MarchArgs<S> A, int *out)
{
    int wid = (int)blockIdx.x;
    if (wid >= A.nwork) return;
    const WorkItem wk = A.work[wid];
    const int lane = (int)(threadIdx.x & 63);
    const LaneStrip ls = FRAMED ? lane_strip(A, wk, lane) : LaneStrip{wk.patch, wk.i0, wk.r0, wk.th, 0};
    const PatchInfo pi = A.patches[ls.patch];
    const int mc = footprint_col<FRAMED>(pi, ls.i0, lane - ls.l0);
    int hot = 0;
    for (int j = 0; j < wk.th + 4; j++) {
        const int k = ls.r0 - 2 + j <= ls.r0 + ls.th + 1 ? ls.r0 - 2 + j : ls.r0 + ls.th + 1;
        const long long idx = footprint_row<FRAMED>(pi, k) + mc;
        hot |= !(relax_c2(A.P, MASK_PHI, (T)A.bath[idx]) > (T)0);
    }
    const int any_hot = __any(hot);
    if (lane == 0) out[wid] = any_hot ? 1 : 0;
}

// class of each item for the coming attempt from the attempt's input mask
// and the bottom part, into cls[wid] (0: no cell the item loads has c^2 =
// 0, so that none of its edges needs the FP64 solve; 1: the others).  One
// wavefront per item.
template <class S, class T, bool FRAMED>
__global__ __launch_bounds__(64) void classify_kernel(MarchArgs<S> A, int *cls)
{
    int wid = (int)blockIdx.x;
    if (wid >= A.nwork) return;
    if (A.latch && *A.latch == 0) return;       // the classes stand (uniform)
    const int lane = (int)(threadIdx.x & 63);
    if (A.clsb[wid]) {                          // uniform over the wavefront
        if (lane == 0) cls[wid] = 1;
        return;
    }
    const WorkItem wk = A.work[wid];
    const LaneStrip ls = FRAMED ? lane_strip(A, wk, lane) : LaneStrip{wk.patch, wk.i0, wk.r0, wk.th, 0};
    const PatchInfo pi = A.patches[ls.patch];
    const uint8_t *mk = A.scen[A.patches[FRAMED ? item_patch(A, wk) : wk.patch].scen].cur ? A.m1 : A.m0;
    const int mc = footprint_col<FRAMED>(pi, ls.i0, lane - ls.l0);
    // loads in batches of ROWS_IN_FLIGHT rows, all issued before any is used
    // (the batches run over the item's tallest tile, a shorter tile's lanes
    // reading their last row again)
    constexpr int ROWS_IN_FLIGHT = 16;
    const int k1 = ls.r0 + ls.th + 1;
    int hot = 0;
    for (int j0 = 0; j0 < wk.th + 4; j0 += ROWS_IN_FLIGHT) {
        int m[ROWS_IN_FLIGHT];
#pragma unroll
        for (int u = 0; u < ROWS_IN_FLIGHT; u++) {
            const int k = ls.r0 - 2 + j0 + u <= k1 ? ls.r0 - 2 + j0 + u : k1;
            m[u] = mk[footprint_row<FRAMED>(pi, k) + mc];
        }
#pragma unroll
        for (int u = 0; u < ROWS_IN_FLIGHT; u++) hot |= (m[u] & (MASK_PHI | MASK_BRK)) != MASK_PHI;
    }
    const int any_hot = __any(hot);
    if (lane == 0) cls[wid] = any_hot ? 1 : 0;
}

// the two item lists from the classes, each in ascending item order, and
// their lengths: one workgroup of NT threads.  The classes are taken in
// passes of 32 x NT items; in a pass thread t holds items p + c NT + t
// (c < 32) as the bits of one word, and an item's place in the list of
// class 1 is the number of class-1 items before it (wave ballots, then a
// scan of the per-wave counts in item order); its place in the other list
// is its index less that number.
constexpr int LIST_THREADS = 1024;

template <int NT>
__global__ __launch_bounds__(NT) void list_kernel(const int *cls, int nwork, int *list,
                                                  unsigned *lcnt, int *latch)
{
    constexpr int NW = NT / 64, CH = 32;
    __shared__ int cnt[CH * NW];        // class-1 counts per (chunk, wave), then their scan
    __shared__ int total;               // class-1 items before the pass
    // no cell latched since the lists were made: they stand (the flag is read
    // by every thread before any barrier, and cleared after the last one)
    if (latch && *latch == 0) return;
    const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) total = 0;
    for (int p = 0; p < nwork; p += CH * NT) {
        unsigned bits = 0;
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int w = p + c * NT + t;
            if (w < nwork && cls[w]) bits |= 1u << c;
        }
        unsigned long long below[CH];   // per chunk: ballot of the lanes below this one
        const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const unsigned long long bal = __ballot((bits >> c) & 1u);
            below[c] = bal & lt;
            if (lane == 0) cnt[c * NW + wave] = __popcll(bal);
        }
        __syncthreads();
        if (wave == 0) {
            // exclusive scan of the CH * NW counts in item order, by lane
            // runs of (CH * NW) / 64 entries, then across lanes
            constexpr int RUN = CH * NW / 64;
            int v[RUN], sum = 0;
#pragma unroll
            for (int r = 0; r < RUN; r++) { v[r] = cnt[lane * RUN + r]; sum += v[r]; }
            int incl = sum;
            for (int o = 1; o < 64; o <<= 1) {
                const int x = __shfl_up(incl, o, 64);
                if (lane >= o) incl += x;
            }
            int run = total + incl - sum;
#pragma unroll
            for (int r = 0; r < RUN; r++) { cnt[lane * RUN + r] = run; run += v[r]; }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CH; c++) {
            const int w = p + c * NT + t;
            if (w < nwork) {
                const int before = cnt[c * NW + wave] + __popcll(below[c]);
                if ((bits >> c) & 1u) list[nwork + before] = w;
                else list[w - before] = w;
            }
        }
        __syncthreads();
        if (t == NT - 1) {
            const int last = cnt[(CH - 1) * NW + NW - 1] + __popcll(below[CH - 1]) + (int)((bits >> (CH - 1)) & 1u);
            total = last;
        }
        __syncthreads();
    }
    if (t == 0) {
        lcnt[0] = (unsigned)(nwork - total);
        lcnt[1] = (unsigned)total;
        if (latch) *latch = 0;
    }
}

}  // namespace hsgn
