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
template <class S, class T, bool MIXED, bool AMR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MIXED ? 2 : 1, MIXED ? 2 : 1)))
void march_kernel(MarchArgs<S> A)
{
    int wid = (int)blockIdx.x;
    if (wid >= A.nwork) return;
    __shared__ T ring[3 * EIG_FIELDS * 64 + (MIXED ? 3 * 7 * 64 : 0)];
    GpuLanes<T> ln{ring};
    march<GpuLanes<T>, S, T, MIXED, AMR>(ln, A, wid);
}


}  // namespace hsgn
