// hsgn_api.hip -- device kernels and the C ABI of the HSGN/SWE step library.
//
// Kernels:
//   march_kernel     one 64-wide wavefront per strip work item advances its
//                    strip by one step (hsgn_march.hpp);
//   control_kernel   per scenario: Courant number from the wavefronts' speed
//                    maxima, accept or reject the attempt, next dt, clock;
//   gauge_kernel     bilinear eta' at the gauges after accepted steps;
//   mask_kernel      transition function phi_T from the bathymetry;
//   initdt_kernel    first adaptive step from the cell speed bound;
//   mass_kernel      FP64 mass per patch in a fixed summation order;
//   count_kernel     SWE and breaking cell counts.
// The host side keeps all device state in one context and never copies
// state between host and device inside hsgn_advance except the per-scenario
// clock records at the end.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <condition_variable>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <thread>

#include <unistd.h>

#include "hsgn.h"
#include "hsgn_amr.hpp"
#include "hsgn_march.hpp"
#include "host_pool.hpp"

using namespace hsgn;

// ---------------------------------------------------------------------------
// device side

// the step kernel is compiled in two translation units with different
// floating-point contraction (hsgn_step64.hip: none, hsgn_step32.hip: FMA)
void launch_march64(const MarchArgs<double> &A, unsigned nwork, hipStream_t stream);
void launch_march32(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream, bool beside);
void launch_march32_deep(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream);
void launch_classify32(const MarchArgs<float> &A, unsigned nwork, int *cls, hipStream_t stream);
void launch_static_class32(const MarchArgs<float> &A, unsigned nwork, int *out, hipStream_t stream);
// instantiations for patches of patch sets (hsgn_step64amr.hip, hsgn_step32amr.hip)
void launch_march64_amr(const MarchArgs<double> &A, unsigned nwork, hipStream_t stream);
void launch_march32_amr(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream, bool beside);
void launch_march32_amr_deep(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream);
void launch_classify32_amr(const MarchArgs<float> &A, unsigned nwork, int *cls, hipStream_t stream);
void launch_static_class32_amr(const MarchArgs<float> &A, unsigned nwork, int *out, hipStream_t stream);

struct ScenStatic {
    double dx, dy, cfl, cfl_max;
    int w0, w1;               // work-item range of the scenario
};

// one block per scenario; the clipped-mass slots are summed in a fixed order
// (strided per thread, then a fixed tree) so results are reproducible
__global__ __launch_bounds__(256) void control_kernel(ScenState *S, const ScenStatic *SS,
                                                      const double *clip_slots, int nscen)
{
    __shared__ double part[256];
    const int s = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    if (s >= nscen) return;
    const ScenStatic ss = SS[s];
    double cs = 0.0;
    for (int w = ss.w0 + tid; w < ss.w1; w += 256) cs += clip_slots[w];
    part[tid] = cs;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) part[tid] += part[tid + h];
        __syncthreads();
    }
    if (tid != 0) return;
    ScenState &st = S[s];
    double rx = __longlong_as_double((long long)st.rx_bits);
    double ry = __longlong_as_double((long long)st.ry_bits);
    st.rx_bits = 0ull;
    st.ry_bits = 0ull;
    st.accepted = 0;
    if (!st.active) return;
    if (st.err != 0) { st.active = 0; return; }
    double dt = st.dt;
    double courant = fmax(dt * rx / ss.dx, dt * ry / ss.dy);
    if (courant > ss.cfl_max) {
        if (!st.adaptive) { st.err = HSGN_ECFL; st.active = 0; return; }
        st.dt = dt * ss.cfl / courant;
        st.rejects += 1;
        st.streak += 1;
        if (st.streak > 64) { st.err = HSGN_ECFL; st.active = 0; }
        return;
    }
    st.streak = 0;
    st.cur ^= 1;
    st.t += dt;
    st.steps += 1;
    st.records += 1;
    st.accepted = 1;
    st.courant = courant;
    st.max_courant = fmax(st.max_courant, courant);
    st.clip_total += part[0];
    if (st.adaptive && courant > 0.0) st.dt = dt * ss.cfl / courant;
    if (st.steps >= st.target) st.active = 0;
}

struct GaugeDev {
    int scen, slot, ng;
    int qscen;                                    // slot whose buffer index the patch uses
    long long qoff, plane, c00, c01, c10, c11;   // cell offsets (bathymetry space)
    double wx, wy;
    long long roff;                               // record area offset
    long long cap;
};

template <class S, bool MIXED>
__global__ void gauge_kernel(const GaugeDev *G, int n, const ScenState *Sc, const S *q0,
                             const S *q1, const S *bath, double eta0, double dry_tol,
                             double *rec)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const GaugeDev g = G[k];
    const ScenState &st = Sc[g.scen];
    if (!st.accepted) return;
    long long r = st.records - 1;
    if (r < 0 || r >= g.cap) return;
    const S *q = Sc[g.qscen].cur ? q1 : q0;
    long long cells[4] = {g.c00, g.c01, g.c10, g.c11};
    double e[4];
    for (int a = 0; a < 4; a++) {
        long long ci = cells[a];
        double v = (double)q[g.qoff + ci];
        double b = (double)bath[g.plane + ci];
        double h = MIXED ? v + eta0 - b : v;
        double ep = MIXED ? v : h + b - eta0;
        e[a] = h > dry_tol ? ep : 0.0;
    }
    double wx = g.wx, wy = g.wy;
    double eta = (1.0 - wx) * (1.0 - wy) * e[0] + wx * (1.0 - wy) * e[1]
               + (1.0 - wx) * wy * e[2] + wx * wy * e[3];
    long long base = g.roff + r * (1 + g.ng);
    if (g.slot == 0) rec[base] = st.t;
    rec[base + 1 + g.slot] = eta;
}

template <class S>
__global__ void mask_kernel(PatchInfo pi, const S *bath, uint8_t *m0, uint8_t *m1,
                            double eta0, double h_star, int n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    double hmin = INFINITY;
    for (int dj = -n; dj <= n; dj++) {
        for (int di = -n; di <= n; di++) {
            int fx, fy;
            // stored ghost cells (patch sets) or the boundary map
            int mx = pi.frame ? x + di : map_index(x + di, pi.nx, pi.bc[0], pi.bc[1], &fx);
            int my = pi.frame ? y + dj : map_index(y + dj, pi.ny, pi.bc[2], pi.bc[3], &fy);
            double H = eta0 - (double)bath[pi.coff + (long long)my * pi.pitch + mx];
            H = H > 0.0 ? H : 0.0;
            hmin = H < hmin ? H : hmin;
        }
    }
    uint8_t phi = hmin > h_star ? 1 : 0;
    long long idx = pi.coff + (long long)y * pi.pitch + x;
    m0[idx] = phi;
    m1[idx] = phi;
}

template <class S, bool MIXED>
__global__ void initdt_kernel(PatchInfo pi, StepParams P, const S *q, const S *bath,
                              const uint8_t *mask, unsigned long long *slot, int *err)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    double m = 0.0;
    if (i < ncell) {
        int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
        long long idx = (long long)y * pi.pitch + x;
        long long plane = pi.plane;
        double b = (double)bath[pi.coff + idx];
        double h = (double)q[pi.qoff + idx];
        if (MIXED) h = h + P.eta0 - b;
        if (h > P.dry_tol) {
            double u = (double)q[pi.qoff + plane + idx] / h, v = (double)q[pi.qoff + 2 * plane + idx] / h;
            double p = (double)q[pi.qoff + 5 * plane + idx] / h;
            uint8_t mk = mask[pi.coff + idx];
            int swe = !(mk & 1) || ((mk >> 1) & 1);
            double H = P.eta0 - b;
            H = H > 0.0 ? H : 0.0;
            double c2 = swe ? 0.0 : P.a2g * H + P.c2f;
            double a = P.g * h + p + c2;
            if (a < 0.0) *err = HSGN_ENONHYP;
            double ce = sqrt(a);
            m = fmax((fabs(u) + ce) / pi.dx, (fabs(v) + ce) / pi.dy);
        }
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(slot, (unsigned long long)__double_as_longlong(m));
}

__global__ void initdt_finish(ScenState *S, const ScenStatic *SS, const unsigned long long *slots,
                              int nscen)
{
    int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= nscen) return;
    double m = __longlong_as_double((long long)slots[s]);
    if (m > 0.0) S[s].dt = SS[s].cfl / m;
    else if (S[s].err == 0) S[s].err = HSGN_EINVAL;
}

// FP64 sum of h (times the capacity on a mapped grid) over one patch: fixed
// decomposition (1024 threads, strided), then a fixed-order tree in shared
// memory
template <class S, bool MIXED>
__global__ __launch_bounds__(1024) void mass_kernel(PatchInfo pi, const S *q, const S *bath,
                                                    double eta0, double *out)
{
    __shared__ double part[1024];
    long long ncell = (long long)pi.nx * pi.ny;
    double s = 0.0;
    for (long long i = threadIdx.x; i < ncell; i += 1024) {
        int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
        long long idx = (long long)y * pi.pitch + x;
        double v = (double)q[pi.qoff + idx];
        if (MIXED) {
            v = v + eta0 - (double)bath[pi.coff + idx];
            v = v > 0.0 ? v : 0.0;
        }
        if (pi.metric) v = v * pi.metric[(long long)(y + 2) * (pi.nx + 4) + (x + 2)];   // capacity
        s += v;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

__global__ void count_kernel(PatchInfo pi, const uint8_t *mask, unsigned long long *cnt)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    uint8_t mk = mask[pi.coff + (long long)y * pi.pitch + x];
    int swe = !(mk & 1) || ((mk >> 1) & 1);
    if (swe) atomicAdd(&cnt[0], 1ull);
    if ((mk >> 1) & 1) atomicAdd(&cnt[1], 1ull);
}

// conversion between the ABI layout (FP64 q[7][ny][nx], plane 0 = h) and the
// stored one (FP64 with plane 0 = h, or FP32 with plane 0 = eta' = h + b -
// eta0; rows of pitch elements, possibly inside a ghost frame)
template <class S, bool MIXED>
__global__ void to_storage_kernel(PatchInfo pi, const double *in, S *q, const S *bath,
                                  double eta0)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    long long idx = (long long)y * pi.pitch + x;
    double b = (double)bath[pi.coff + idx];
    q[pi.qoff + idx] = MIXED ? (S)(in[i] + b - eta0) : (S)in[i];
    for (int m = 1; m < 7; m++) q[pi.qoff + m * pi.plane + idx] = (S)in[m * ncell + i];
}

template <class S, bool MIXED>
__global__ void from_storage_kernel(PatchInfo pi, const S *q, const S *bath, double eta0,
                                    double *out)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    long long idx = (long long)y * pi.pitch + x;
    if (MIXED) {
        double b = (double)bath[pi.coff + idx];
        double h = (double)q[pi.qoff + idx] + eta0 - b;
        out[i] = h > 0.0 ? h : 0.0;
    } else {
        out[i] = (double)q[pi.qoff + idx];
    }
    for (int m = 1; m < 7; m++) out[m * ncell + i] = (double)q[pi.qoff + m * pi.plane + idx];
}

// mixed storage under a new bottom bnew (ABI layout, FP64): eta' of every
// interior cell of the patch becomes h + bnew - eta0, with h from the old
// bottom, so that the depth is kept (the new bottom is stored in FP32)
__global__ void keep_depth_kernel(PatchInfo pi, float *q, const float *bath, const double *bnew,
                                  double eta0)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    long long idx = (long long)y * pi.pitch + x;
    const double h = (double)q[pi.qoff + idx] + eta0 - (double)bath[pi.coff + idx];
    q[pi.qoff + idx] = (float)(h + (double)(float)bnew[i] - eta0);
}

// one cell plane (bathymetry or mask) between the ABI layout and storage
template <class A, class S>
__global__ void scatter_plane_kernel(PatchInfo pi, const A *in, S *out, int keep_high_bits)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    long long idx = pi.coff + (long long)y * pi.pitch + x;
    if (keep_high_bits) out[idx] = (S)(((int)out[idx] & ~3) | ((int)in[i] & 3));
    else out[idx] = (S)in[i];
}

// the bathymetry of many patches from one host-order buffer: records of
// (patch, first cell) sorted by their first cell
struct BulkRec {
    PatchInfo p;
    long long c0;
};

template <class S>
__global__ void scatter_bulk_kernel(const BulkRec *R, int nr, long long total, const double *in,
                                    S *out)
{
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (R[mid].c0 <= k) lo = mid;
        else hi = mid - 1;
    }
    const PatchInfo pi = R[lo].p;
    const long long e = k - R[lo].c0;
    const int x = (int)(e % pi.nx), y = (int)(e / pi.nx);
    out[pi.coff + (long long)y * pi.pitch + x] = (S)in[k];
}

// phi_T of many patch-set patches at once (records as for scatter_bulk_kernel)
template <class S>
__global__ void mask_bulk_kernel(const BulkRec *R, int nr, long long total, const S *bath,
                                 uint8_t *m0, uint8_t *m1, double eta0, double h_star, int n)
{
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (R[mid].c0 <= k) lo = mid;
        else hi = mid - 1;
    }
    const PatchInfo pi = R[lo].p;
    const long long e = k - R[lo].c0;
    const int x = (int)(e % pi.nx), y = (int)(e / pi.nx);
    double hmin = INFINITY;
    for (int dj = -n; dj <= n; dj++)
        for (int di = -n; di <= n; di++) {
            double H = eta0 - (double)bath[pi.coff + (long long)(y + dj) * pi.pitch + (x + di)];
            H = H > 0.0 ? H : 0.0;
            hmin = H < hmin ? H : hmin;
        }
    const uint8_t phi = hmin > h_star ? 1 : 0;
    const long long idx = pi.coff + (long long)y * pi.pitch + x;
    m0[idx] = phi;
    m1[idx] = phi;
}

template <class S, class A>
__global__ void gather_plane_kernel(PatchInfo pi, const S *in, A *out, int low_bits_only)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    S v = in[pi.coff + (long long)y * pi.pitch + x];
    out[i] = low_bits_only ? (A)((int)v & 3) : (A)v;
}

__global__ void to_float_kernel(const double *in, float *out, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// host side

struct ScenHost {
    std::vector<int> patches;              // every patch of the scenario, in add order
    std::vector<std::vector<int>> lev;     // patch ids per refinement level
    std::vector<int> slot;                 // clock slot of each level (slot[0] = scenario)
    bool amr = false;                      // more than one patch: a patch set
    int NX = 0, NY = 0;                    // level-0 domain size in cells (patch sets)
    double X0 = 0.0, Y0 = 0.0;             // domain corner
    int bc[4] = {0, 0, 0, 0};              // domain boundary conditions (patch sets)
    std::vector<double> gauge_xy;
    long long gcap = 0, roff = 0;
    int ng = 0;
    double sp_w[4] = {0.0, 0.0, 0.0, 0.0};  // sponge widths (m) and peak rate (1/s)
    double sp_rate = 0.0;
};

// table ranges of one refinement level
struct LevelRange {
    int w0 = 0, w1 = 0, wa = 0;     // work items [w0, w1); [w0, wa) single-grid, [wa, w1) patch sets
    int s0 = 0, s1 = 0;             // clock slots
    int gc0 = 0, gc1 = 0;           // ghost copies
    int gi0 = 0, gi1 = 0;           // ghost interpolations
    int fr0 = 0, fr1 = 0;           // boundary-flux records (this level as the fine one)
    int rf0 = 0, rf1 = 0;           // reflux records (this level as the coarse one)
    int av0 = 0, av1 = 0;           // average-down records (this level as the fine one)
    long long e0 = 0, e1 = 0;       // boundary-flux entries (7-vectors)
};

// host memory of the tables below: pinned, so that uploads run as direct
// transfers; where pinning fails, ordinary memory, remembered here so that it
// is freed the same way (HSGN_PAGEABLE_TABLES=1 takes ordinary memory
// always: a diagnostic, results are the same bit for bit)
struct TableMemory {
    static void *get(size_t bytes)
    {
        void *p = nullptr;
        const char *pageable = getenv("HSGN_PAGEABLE_TABLES");
        if (!(pageable && pageable[0] == '1')) {
            if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess && p) return p;
            (void)hipGetLastError();        // the failure must not reach a later check
        }
        p = ::operator new(bytes);
        std::lock_guard<std::mutex> lk(m());
        plain().insert(p);
        return p;
    }
    static void put(void *p)
    {
        {
            std::lock_guard<std::mutex> lk(m());
            auto it = plain().find(p);
            if (it != plain().end()) {
                plain().erase(it);
                ::operator delete(p);
                return;
            }
        }
        (void)hipHostFree(p);
    }
    // never torn down: a table may be freed late in the process's exit
    static std::mutex &m()
    {
        static std::mutex *x = new std::mutex();
        return *x;
    }
    static std::set<void *> &plain()
    {
        static std::set<void *> *x = new std::set<void *>();
        return *x;
    }
};

// host tables that are sized first and then filled: resize() leaves the new
// records uninitialised instead of zeroing them.  A regrid hands the old
// context's tables to the new context, which reuses their memory.
template <class T>
struct DefaultInitAlloc {
    using value_type = T;
    template <class U> struct rebind { using other = DefaultInitAlloc<U>; };
    DefaultInitAlloc() = default;
    template <class U> DefaultInitAlloc(const DefaultInitAlloc<U> &) noexcept {}
    T *allocate(size_t n) { return static_cast<T *>(TableMemory::get(n * sizeof(T))); }
    void deallocate(T *p, size_t) noexcept { TableMemory::put(p); }
    template <class U> void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value)
    {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... A> void construct(U *p, A &&...a)
    {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
    template <class U> bool operator==(const DefaultInitAlloc<U> &) const noexcept { return true; }
    template <class U> bool operator!=(const DefaultInitAlloc<U> &) const noexcept { return false; }
};
template <class T> using HostVec = std::vector<T, DefaultInitAlloc<T>>;

struct hsgn_ctx {
    hsgn_params prm;
    StepParams P;
    hipStream_t stream = nullptr;
    bool finalized = false;
    std::vector<PatchInfo> patches;
    std::vector<std::vector<double>> braw;   // bathymetry as set, per patch (host copy)
    double *d_B0 = nullptr;     // device level-0 bathymetry of scenario b0_scen (regridding)
    int b0_scen = -1;
    std::vector<char> braw_rule;             // 1: a regridded patch, bathymetry from the
                                             // level-0 bathymetry (no host copy kept)
    std::vector<double> px0, py0;
    std::vector<int> pI0, pJ0;             // patch origin in cells of its level (patch sets)
    std::vector<ScenHost> scen;
    std::vector<WorkItem> work;
    std::vector<PackedItem> packs;            // strips of the packed items
    std::vector<ScenStatic> sstat;
    int nslot = 0, nlev = 1;
    bool any_amr = false;
    std::vector<int> slot_scen, slot_level;   // scenario and level of each clock slot
    std::vector<int> th_level;                // tile rows per refinement level
    std::vector<LevelRange> L;
    bool mixed = false;         // FP32 eta' storage with FP64 near-shore edges
    // device (FP64 storage: q0, q1, bath; mixed storage: f0, f1, fbath)
    double *q0 = nullptr, *q1 = nullptr, *bath = nullptr, *clip = nullptr, *rec = nullptr;
    float *f0 = nullptr, *f1 = nullptr, *fbath = nullptr;
    double *stage = nullptr;    // FP64 staging for conversions at the ABI
    void *arena = nullptr;      // one allocation holding the buffers fixed at finalize
    long long stage_len = 0;
    uint8_t *m0 = nullptr, *m1 = nullptr;
    PatchInfo *d_patches = nullptr;
    WorkItem *d_work = nullptr;
    PackedItem *d_packs = nullptr;
    int *d_list = nullptr;      // item lists of the split mixed step (2 per item)
    unsigned *d_lcnt = nullptr; // their lengths
    int *d_cls = nullptr;       // the items' classes for the attempt
    int *d_latch = nullptr;     // split step over single grids only: a cell latched since
                                // the lists were made (1 forces the classification)
    std::vector<uint8_t> state_set;   // per patch: its state has been set (or moved in)
    uint8_t *d_keep = nullptr;  // device copy of state_set for the bathymetry average-down
    int *d_clsb = nullptr;      // their bottom part
    bool clsb_dirty = true;     // d_clsb to recompute (bathymetry or work table changed)
    bool split = false;         // mixed single grids: deep items without the FP64 edges
    bool pack = true;           // patch sets: narrow strips packed into shared wavefronts
    bool any_sponge = false;    // some scenario has a sponge (step kernels with it)
    bool any_mapped = false;    // some patch is mapped
    bool mapped_single = false; // some single grid is mapped: the single-grid
                                // launches take the mapped step kernel
    bool mapped_amr = false;    // the same for the patch-set launches
    std::vector<double *> d_metric;   // per patch: its metric planes, or null
    ScenState *d_scen = nullptr;
    ScenStatic *d_sstat = nullptr;
    GaugeDev *d_gauges = nullptr;
    unsigned long long *d_slots = nullptr;
    unsigned long long *d_cnt = nullptr;
    int *d_err = nullptr;
    double *d_mass = nullptr;
    int ngauge_total = 0;
    long long qtotal = 0, ctotal = 0, rec_total = 0;
    // patch sets
    HostVec<GhostCopy> h_gc;
    HostVec<GhostInterp> h_gi;
    HostVec<FluxRec> h_fr;
    std::vector<RefluxRec> h_rf;
    HostVec<AvgRec> h_av;
    int ngc = 0, ngi = 0;           // ghost copy and interpolation records on the device
    GhostCopy *d_gc = nullptr;
    GhostInterp *d_gi = nullptr;
    FluxRec *d_fr = nullptr;
    RefluxRec *d_rf = nullptr;
    AvgRec *d_av = nullptr;
    double *d_E = nullptr, *d_R = nullptr, *d_rclip = nullptr;
    long long etotal = 0;
    bool amr_dirty = true;
    hipStream_t cap_stream = nullptr;
    hipStream_t aux_stream = nullptr;           // items of the split step that need FP64 edges
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false, graph_failed = false;
    std::string last_error;
    // optional step-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;     // pairs (start, stop) per timed launch
    size_t ev_used = 0;
    double timed_ms = 0.0;
    long long timed_launches = 0;
};

static int fail(hsgn_ctx *c, int code, const std::string &msg)
{
    if (c) c->last_error = msg;
    return code;
}

#define HIPCHK(c, expr)                                                            \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail((c), HSGN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static void free_events(hsgn_ctx *c)
{
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    c->ev_used = 0;
}

static void drop_graph(hsgn_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->graph_valid = false;
}

static void free_device(hsgn_ctx *c)
{
    free_events(c);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    c->aux_stream = nullptr;
    c->ev_fork = c->ev_join = nullptr;
    // the buffers fixed at finalize go with the arena
    void *ptrs[] = {c->arena, c->clip, c->rec, c->d_work, c->d_gauges, c->d_list, c->d_clsb,
                    c->d_cls, c->d_B0, c->d_packs};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (double *m : c->d_metric)
        if (m) (void)hipFree(m);
    c->d_metric.clear();
    c->q0 = c->q1 = c->bath = c->clip = c->rec = c->d_mass = c->stage = nullptr;
    c->f0 = c->f1 = c->fbath = nullptr;
    c->m0 = c->m1 = nullptr;
    c->d_patches = nullptr; c->d_work = nullptr; c->d_scen = nullptr; c->d_sstat = nullptr;
    c->d_gauges = nullptr; c->d_slots = nullptr; c->d_err = nullptr; c->d_cnt = nullptr;
    c->d_gc = nullptr; c->d_gi = nullptr; c->d_fr = nullptr; c->d_rf = nullptr; c->d_av = nullptr;
    c->d_E = c->d_R = c->d_rclip = nullptr;
    c->d_list = c->d_clsb = c->d_cls = nullptr;
    c->d_keep = nullptr;
    c->d_B0 = nullptr;
    c->d_packs = nullptr;
    c->d_latch = nullptr;
    c->arena = nullptr;
    c->b0_scen = -1;
    c->d_lcnt = nullptr;
}

template <class S>
static MarchArgs<S> march_args(hsgn_ctx *c, S *q0, S *q1, const S *bath, int w0, int w1)
{
    MarchArgs<S> A;
    A.P = c->P;
    A.patches = c->d_patches;
    A.work = c->d_work + w0;
    A.packs = c->d_packs;
    A.q0 = q0; A.q1 = q1;
    A.bath = bath;
    A.m0 = c->m0; A.m1 = c->m1;
    A.scen = c->d_scen;
    A.clip_slots = c->clip + w0;
    A.eflux = c->d_E;
    A.list = nullptr;
    A.lcnt = nullptr;
    A.clsb = nullptr;
    A.latch = nullptr;
    A.sponge = c->any_sponge ? 1 : 0;
    A.mapped = c->mapped_single ? 1 : 0;   // patch-set ranges: launch_march_range
    A.nwork = w1 - w0;
    return A;
}

template <class S>
static AmrBuffers<S> amr_buffers(hsgn_ctx *c, S *q0, S *q1, S *bath)
{
    AmrBuffers<S> B;
    B.patches = c->d_patches;
    B.scen = c->d_scen;
    B.q0 = q0; B.q1 = q1;
    B.bath = bath;
    B.m0 = c->m0; B.m1 = c->m1;
    return B;
}

// ---------------------------------------------------------------------------
// host worker threads (host_pool.hpp)

static int host_threads() { return HostPool::get().size(); }

// ---------------------------------------------------------------------------
// patch-set geometry: which patch of a level covers a cell

struct LevelIndex {
    static constexpr int BS = 64;                     // bucket side in cells
    std::vector<std::vector<int>> buckets;            // dense over the level's domain
    long long NXl = 0, NYl = 0, nbx = 0, nby = 0;
    const hsgn_ctx *c = nullptr;
    static long long fdiv(long long a, long long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
    void init(const hsgn_ctx *ctx, long long nx, long long ny)
    {
        c = ctx;
        NXl = nx; NYl = ny;
        nbx = (nx + BS - 1) / BS;
        nby = (ny + BS - 1) / BS;
        buckets.assign((size_t)(nbx * nby), std::vector<int>());
    }
    void add(int pid)
    {
        const PatchInfo &p = c->patches[pid];
        long long I0 = c->pI0[pid], J0 = c->pJ0[pid];
        long long b0 = std::max(fdiv(J0, BS), 0LL), b1 = std::min(fdiv(J0 + p.ny - 1, BS), nby - 1);
        long long a0 = std::max(fdiv(I0, BS), 0LL), a1 = std::min(fdiv(I0 + p.nx - 1, BS), nbx - 1);
        for (long long bj = b0; bj <= b1; bj++)
            for (long long bi = a0; bi <= a1; bi++) buckets[(size_t)(bj * nbx + bi)].push_back(pid);
    }
    // the patches of the buckets that cells [I0, I0 + nx) x [J0, J0 + ny)
    // reach, with repeats
    void near(long long I0, long long J0, long long nx, long long ny, std::vector<int> &out) const
    {
        long long b0 = std::max(fdiv(J0, BS), 0LL), b1 = std::min(fdiv(J0 + ny - 1, BS), nby - 1);
        long long a0 = std::max(fdiv(I0, BS), 0LL), a1 = std::min(fdiv(I0 + nx - 1, BS), nbx - 1);
        for (long long bj = b0; bj <= b1; bj++)
            for (long long bi = a0; bi <= a1; bi++)
                for (int pid : buckets[(size_t)(bj * nbx + bi)]) out.push_back(pid);
    }
    int find(long long I, long long J) const
    {
        if (I < 0 || J < 0 || I >= NXl || J >= NYl) return -1;
        for (int pid : buckets[(size_t)((J / BS) * nbx + I / BS)]) {
            const PatchInfo &p = c->patches[pid];
            long long I0 = c->pI0[pid], J0 = c->pJ0[pid];
            if (I >= I0 && I < I0 + p.nx && J >= J0 && J < J0 + p.ny) return pid;
        }
        return -1;
    }
    // the same, trying the patch of the caller's last hit first (patches of
    // a level do not overlap and lie inside its domain: the answer is the
    // same)
    int find(long long I, long long J, int &hint) const
    {
        if (hint >= 0) {
            const PatchInfo &p = c->patches[hint];
            long long I0 = c->pI0[hint], J0 = c->pJ0[hint];
            if (I >= I0 && I < I0 + p.nx && J >= J0 && J < J0 + p.ny) return hint;
        }
        const int pid = find(I, J);
        if (pid >= 0) hint = pid;
        return pid;
    }
};

static int host_map(int i, int n, int lo, int hi, int *flip)
{
    *flip = 0;
    if (i < 0) {
        if (lo == HSGN_BC_PERIODIC) return i + n;
        if (lo == HSGN_BC_WALL) { *flip = 1; return -1 - i; }
        return 0;
    }
    if (i >= n) {
        if (hi == HSGN_BC_PERIODIC) return i - n;
        if (hi == HSGN_BC_WALL) { *flip = 1; return 2 * n - 1 - i; }
        return n - 1;
    }
    return i;
}

static int local_of(const PatchInfo &p, long long i, long long j) { return (int)(j * p.pitch + i); }

// validate a patch set and build its tables (appended to the context's)
// per patch of a patch set: its ghost, boundary-flux and covered-cell records
struct PatchRecs {
    std::vector<GhostCopy> gc;
    std::vector<GhostInterp> gi;
    std::vector<FluxRec> fr;
    std::vector<AvgRec> av;
    const char *err = nullptr;
};

// the tables of patch-set scenario s, appended per level: lev_recs[l] gets
// the records of its level-l patches in patch order, lev_rf[l] its reflux
// records in (J, I) order
static int build_patch_set(hsgn_ctx *c, int s, std::vector<std::vector<PatchRecs>> &lev_recs,
                           std::vector<std::vector<RefluxRec>> &lev_rf)
{
    ScenHost &sh = c->scen[s];
    const int nl = (int)sh.lev.size();
    std::vector<LevelIndex> idx(nl);
    for (int l = 0; l < nl; l++) {
        long long f = 1;
        for (int k = 0; k < l; k++) f *= AMR_RATIO;
        idx[l].init(c, (long long)sh.NX * f, (long long)sh.NY * f);
        for (int pid : sh.lev[l]) idx[l].add(pid);
    }
    // finer patches stay one coarser cell away from the domain boundary
    for (int l = 1; l < nl; l++) {
        long long NXl = (long long)sh.NX, NYl = (long long)sh.NY;
        for (int k = 0; k < l; k++) { NXl *= AMR_RATIO; NYl *= AMR_RATIO; }
        for (int pid : sh.lev[l]) {
            const PatchInfo &p = c->patches[pid];
            if (c->pI0[pid] < AMR_RATIO || c->pJ0[pid] < AMR_RATIO ||
                c->pI0[pid] + p.nx > NXl - AMR_RATIO || c->pJ0[pid] + p.ny > NYl - AMR_RATIO)
                return fail(c, HSGN_EINVAL, "a refined patch touches the domain boundary");
        }
    }
    // no two patches of a level overlap.  Every patch lies inside its level's
    // domain (level 0 spans its patches' extent, finer levels were checked
    // above), so two patches that overlap share a bucket of the index.
    for (int l = 0; l < nl; l++)
        for (const std::vector<int> &b : idx[l].buckets)
            for (size_t u = 0; u < b.size(); u++)
                for (size_t v = u + 1; v < b.size(); v++) {
                    const int pid = b[u], q = b[v];
                    const PatchInfo &p = c->patches[pid], &o = c->patches[q];
                    bool ov = c->pI0[pid] < c->pI0[q] + o.nx && c->pI0[q] < c->pI0[pid] + p.nx &&
                              c->pJ0[pid] < c->pJ0[q] + o.ny && c->pJ0[q] < c->pJ0[pid] + p.ny;
                    if (ov) return fail(c, HSGN_EINVAL, "patches of one level overlap");
                }
    long long area = 0;
    for (int pid : sh.lev[0]) area += (long long)c->patches[pid].nx * c->patches[pid].ny;
    if (area != (long long)sh.NX * sh.NY)
        return fail(c, HSGN_EINVAL, "level-0 patches must tile a rectangle");
    // per patch: ghost, boundary-flux and covered-cell records.  Patches are
    // independent (the indexes are read only), so they are built on host
    // threads and kept in patch order: the tables do not depend on the
    // number of threads.
    auto build_one = [&](int l, int pid, PatchRecs &out) {
        const PatchInfo &P = c->patches[pid];
        const long long I0 = c->pI0[pid], J0 = c->pJ0[pid];
        int h_same = -1, h_coarse[5] = {-1, -1, -1, -1, -1};      // last hits of find
        // ghost cells
        for (int j = -2; j < P.ny + 2; j++)
            for (int i = -2; i < P.nx + 2; i++) {
                if (i >= 0 && i < P.nx && j >= 0 && j < P.ny) continue;
                long long I = I0 + i, J = J0 + j;
                if (l == 0) {
                    int fx, fy;
                    int mi = host_map((int)I, sh.NX, sh.bc[0], sh.bc[1], &fx);
                    int mj = host_map((int)J, sh.NY, sh.bc[2], sh.bc[3], &fy);
                    int sp = idx[0].find(mi, mj, h_same);
                    if (sp < 0) { out.err = "level-0 patches leave a hole"; return; }
                    // mapped walls: the domain edge of the source cell's row
                    // (x) or column (y), as the left (bottom) edge of a cell
                    // of the source patch's frame
                    const PatchInfo &Sp = c->patches[sp];
                    const long long wi = (I < 0 ? 0 : sh.NX) - c->pI0[sp];
                    const long long wj = (J < 0 ? 0 : sh.NY) - c->pJ0[sp];
                    out.gc.push_back({pid, local_of(P, i, j), sp,
                                      local_of(Sp, mi - c->pI0[sp], mj - c->pJ0[sp]),
                                      fx | (fy << 1),
                                      fx ? local_of(Sp, wi, mj - c->pJ0[sp]) : 0,
                                      fy ? local_of(Sp, mi - c->pI0[sp], wj) : 0});
                    continue;
                }
                int sp = idx[l].find(I, J, h_same);
                if (sp >= 0) {
                    out.gc.push_back({pid, local_of(P, i, j), sp,
                                      local_of(c->patches[sp], I - c->pI0[sp], J - c->pJ0[sp]), 0,
                                      0, 0});
                    continue;
                }
                long long Ic = LevelIndex::fdiv(I, AMR_RATIO), Jc = LevelIndex::fdiv(J, AMR_RATIO);
                GhostInterp g;
                g.dp = pid;
                g.dl = local_of(P, i, j);
                const long long nb[5][2] = {{Ic, Jc}, {Ic - 1, Jc}, {Ic + 1, Jc}, {Ic, Jc - 1}, {Ic, Jc + 1}};
                for (int k = 0; k < 5; k++) {
                    int cp = idx[l - 1].find(nb[k][0], nb[k][1], h_coarse[k]);
                    g.cp[k] = cp;
                    g.cl[k] = cp >= 0 ? local_of(c->patches[cp], nb[k][0] - c->pI0[cp],
                                                 nb[k][1] - c->pJ0[cp]) : 0;
                }
                if (g.cp[0] < 0) { out.err = "refined patch not properly nested"; return; }
                g.ox = (float)(((double)(I - AMR_RATIO * Ic) + 0.5) / AMR_RATIO - 0.5);
                g.oy = (float)(((double)(J - AMR_RATIO * Jc) + 0.5) / AMR_RATIO - 0.5);
                out.gi.push_back(g);
            }
        if (l == 0) return;
        // boundary edges facing the coarser level: left, right, bottom, top
        for (int side = 0; side < 4; side++) {
            int len = side < 2 ? P.ny : P.nx;
            for (int k = 0; k < len; k++) {
                int gi_ = side == 0 ? -1 : side == 1 ? P.nx : k;
                int gj_ = side < 2 ? k : side == 2 ? -1 : P.ny;
                long long I = I0 + gi_, J = J0 + gj_;
                if (idx[l].find(I, J, h_same) >= 0) continue;
                long long Ic = LevelIndex::fdiv(I, AMR_RATIO), Jc = LevelIndex::fdiv(J, AMR_RATIO);
                int cp = idx[l - 1].find(Ic, Jc, h_coarse[0]);
                if (cp < 0) { out.err = "refined patch not properly nested"; return; }
                int entry = side == 0 ? k : side == 1 ? P.ny + k : side == 2 ? 2 * P.ny + k
                                                                               : 2 * P.ny + P.nx + k;
                out.fr.push_back({pid, entry, local_of(P, gi_, gj_), cp,
                                  local_of(c->patches[cp], Ic - c->pI0[cp], Jc - c->pJ0[cp]),
                                  side < 2 ? 0 : 1, (side == 0 || side == 2) ? 1 : 0});
            }
        }
        // covered coarse cells
        for (int jj = 0; jj < P.ny / AMR_RATIO; jj++)
            for (int ii = 0; ii < P.nx / AMR_RATIO; ii++) {
                long long Ic = I0 / AMR_RATIO + ii, Jc = J0 / AMR_RATIO + jj;
                int cp = idx[l - 1].find(Ic, Jc, h_coarse[0]);
                if (cp < 0) { out.err = "refined patch outside the coarser level"; return; }
                out.av.push_back({pid, local_of(P, AMR_RATIO * ii, AMR_RATIO * jj), cp,
                                  local_of(c->patches[cp], Ic - c->pI0[cp], Jc - c->pJ0[cp])});
            }
    };
    const int nthreads = host_threads();
    for (int l = 0; l < nl; l++) {
        const std::vector<int> &L = sh.lev[l];
        std::vector<PatchRecs> recs(L.size());
        // one task per patch (patches differ in size; the workers take them
        // as they come free)
        if (L.size() > 8)
            HostPool::get().parallel_for((int)L.size(), [&](int k) { build_one(l, L[k], recs[k]); });
        else
            for (size_t k = 0; k < L.size(); k++) build_one(l, L[k], recs[k]);
        for (auto &r : recs)
            if (r.err) return fail(c, HSGN_EINVAL, r.err);
        for (auto &r : recs) lev_recs[l].push_back(std::move(r));
    }
    for (int l = 0; l < nl; l++) {
        // reflux records: uncovered level-l cells next to a level-(l+1) patch
        if (l + 1 < nl) {
            // candidate cells: the ring of level-l cells around each finer
            // patch (inside the domain: finer patches stay one cell away from
            // its boundary), sorted in (J, I) order without repeats.  Small
            // levels mark them in a bitmap read back row by row; large ones
            // sort the list.
            std::vector<std::pair<long long, long long>> cand;
            const long long NXl = idx[l].NXl, NYl = idx[l].NYl;
            const long long words = (NXl + 63) / 64;
            const bool bitmap = words * NYl <= (1LL << 24);         // at most 128 MB
            std::vector<uint64_t> mark(bitmap ? (size_t)(words * NYl) : 0, 0);
            std::vector<uint8_t> row_used(bitmap ? (size_t)NYl : 0, 0);
            auto put = [&](long long J, long long I) {
                if (!bitmap) { cand.push_back({J, I}); return; }
                if (I < 0 || J < 0 || I >= NXl || J >= NYl) return;
                mark[(size_t)(J * words + I / 64)] |= 1ull << (I % 64);
                row_used[(size_t)J] = 1;
            };
            for (int f : sh.lev[l + 1]) {
                const PatchInfo &F = c->patches[f];
                long long a0 = c->pI0[f] / AMR_RATIO, b0 = c->pJ0[f] / AMR_RATIO;
                long long a1 = a0 + F.nx / AMR_RATIO, b1 = b0 + F.ny / AMR_RATIO;
                for (long long J = b0; J < b1; J++) { put(J, a0 - 1); put(J, a1); }
                for (long long I = a0; I < a1; I++) { put(b0 - 1, I); put(b1, I); }
            }
            if (bitmap) {
                for (long long J = 0; J < NYl; J++) {
                    if (!row_used[(size_t)J]) continue;
                    for (long long w = 0; w < words; w++) {
                        uint64_t m = mark[(size_t)(J * words + w)];
                        while (m) {
                            const int b = __builtin_ctzll(m);
                            cand.push_back({J, w * 64 + b});
                            m &= m - 1;
                        }
                    }
                }
            } else {
                std::sort(cand.begin(), cand.end());
                cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            }
            // the records of the candidates, in chunks on host threads joined
            // in order
            const size_t ncand = cand.size();
            const int nt = ncand >= 4096 ? 4 * nthreads : 1;
            std::vector<std::vector<RefluxRec>> part(nt);
            auto reflux_chunk = [&](int t) {
                int h_c = -1, h_f = -1, h_cov = -1;               // last hits of find
                auto covered_h = [&](long long I, long long J) {
                    return idx[l + 1].find(AMR_RATIO * I, AMR_RATIO * J, h_cov) >= 0;
                };
                for (size_t kc = ncand * t / nt; kc < ncand * (t + 1) / nt; kc++) {
                    long long J = cand[kc].first, I = cand[kc].second;
                    int cp = idx[l].find(I, J, h_c);
                    if (cp < 0 || covered_h(I, J)) continue;
                    RefluxRec r;
                    r.cp = cp;
                    r.cl = local_of(c->patches[cp], I - c->pI0[cp], J - c->pJ0[cp]);
                    const long long nb[4][2] = {{I - 1, J}, {I + 1, J}, {I, J - 1}, {I, J + 1}};
                    bool any = false;
                    for (int e = 0; e < 4; e++) {
                        r.fp[e] = -1;
                        r.e0[e] = 0;
                        if (!covered_h(nb[e][0], nb[e][1])) continue;
                        // a fine cell just across the edge
                        long long fi = e == 0 ? AMR_RATIO * I - 1
                                     : e == 1 ? AMR_RATIO * (I + 1) : AMR_RATIO * I;
                        long long fj = e == 2 ? AMR_RATIO * J - 1
                                     : e == 3 ? AMR_RATIO * (J + 1) : AMR_RATIO * J;
                        int f = idx[l + 1].find(fi, fj, h_f);
                        const PatchInfo &F = c->patches[f];
                        long long fI0 = c->pI0[f], fJ0 = c->pJ0[f];
                        r.fp[e] = f;
                        r.e0[e] = e == 0 ? (int)(F.ny + AMR_RATIO * J - fJ0)
                                : e == 1 ? (int)(AMR_RATIO * J - fJ0)
                                : e == 2 ? (int)(2 * F.ny + F.nx + AMR_RATIO * I - fI0)
                                         : (int)(2 * F.ny + AMR_RATIO * I - fI0);
                        any = true;
                    }
                    if (any) part[t].push_back(r);
                }
            };
            HostPool::get().parallel_for(nt, reflux_chunk);
            for (auto &v : part) lev_rf[l].insert(lev_rf[l].end(), v.begin(), v.end());
        }
    }
    return HSGN_OK;
}

// every table entry addresses cells inside its patch's storage (interior or
// ghost frame as required) and entries inside the flux buffer: checked on
// the host before any kernel reads a table
// the cell (i, j) that a local index of a patch addresses (false: before the
// patch's storage); 32-bit division where the storage allows it
static bool cell_of(const PatchInfo &p, int local, long long &i, long long &j)
{
    const long long base = (long long)local + (long long)p.frame * p.pitch + p.frame;
    if (base < 0) return false;
    if (base <= INT_MAX && p.pitch <= INT_MAX) {
        const int b = (int)base, w = (int)p.pitch;
        i = b % w - p.frame;
        j = b / w - p.frame;
    } else {
        i = base % p.pitch - p.frame;
        j = base / p.pitch - p.frame;
    }
    return true;
}

static bool local_ok(const hsgn_ctx *c, int pid, int local, bool interior)
{
    if (pid < 0 || pid >= (int)c->patches.size()) return false;
    const PatchInfo &p = c->patches[pid];
    long long i, j;
    if (!cell_of(p, local, i, j)) return false;
    if (interior) return i >= 0 && i < p.nx && j >= 0 && j < p.ny;
    return i >= -p.frame && i < p.nx + p.frame && j >= -p.frame && j < p.ny + p.frame &&
           !(i >= 0 && i < p.nx && j >= 0 && j < p.ny);
}

// true if ok(k) holds for every k < n, checked on host threads
template <class F>
static bool all_of_parallel(size_t n, F ok)
{
    const int nt = n < 4096 ? 1 : host_threads();
    std::vector<char> good(nt, 1);
    HostPool::get().parallel_for(nt, [&](int t) {
        for (size_t k = (size_t)t; k < n; k += (size_t)nt)
            if (!ok(k)) { good[t] = 0; return; }
    });
    for (char g : good)
        if (!g) return false;
    return true;
}

// the first kind of record that fails the check, or null
static const char *table_error(const hsgn_ctx *c)
{
    // a cell of a patch's frame (interior or ghost), for the wall edges
    auto in_frame = [&](int pid, int local) {
        const PatchInfo &p = c->patches[pid];
        long long i, j;
        return cell_of(p, local, i, j) && i >= -p.frame && i < p.nx + p.frame &&
               j >= -p.frame && j < p.ny + p.frame;
    };
    if (!all_of_parallel(c->h_gc.size(), [&](size_t k) {
            const GhostCopy &r = c->h_gc[k];
            return local_ok(c, r.dp, r.dl, false) && local_ok(c, r.sp, r.sl, true) &&
                   (!(r.flips & 1) || in_frame(r.sp, r.wx)) && (!(r.flips & 2) || in_frame(r.sp, r.wy));
        }))
        return "ghost copy";
    if (!all_of_parallel(c->h_gi.size(), [&](size_t k) {
            const GhostInterp &r = c->h_gi[k];
            if (!local_ok(c, r.dp, r.dl, false) || r.cp[0] < 0) return false;
            for (int s = 0; s < 5; s++)
                if (r.cp[s] >= 0 && !local_ok(c, r.cp[s], r.cl[s], true)) return false;
            return true;
        }))
        return "ghost interpolation";
    if (!all_of_parallel(c->h_fr.size(), [&](size_t k) {
            const FluxRec &r = c->h_fr[k];
            if (!local_ok(c, r.fp, r.gl, false) || !local_ok(c, r.cp, r.cl, true)) return false;
            const PatchInfo &F = c->patches[r.fp];
            return !(F.eoff < 0 || r.entry < 0 || r.entry >= 2 * (F.nx + F.ny));
        }))
        return "flux record";
    if (!all_of_parallel(c->h_rf.size(), [&](size_t k) {
            const RefluxRec &r = c->h_rf[k];
            if (!local_ok(c, r.cp, r.cl, true)) return false;
            for (int e = 0; e < 4; e++) {
                if (r.fp[e] < 0) continue;
                if (r.fp[e] >= (int)c->patches.size()) return false;
                const PatchInfo &F = c->patches[r.fp[e]];
                int lo = e == 0 ? F.ny : e == 1 ? 0 : e == 2 ? 2 * F.ny + F.nx : 2 * F.ny;
                int len = e < 2 ? F.ny : F.nx;
                if (F.eoff < 0 || r.e0[e] < lo || r.e0[e] + AMR_RATIO > lo + len) return false;
            }
            return true;
        }))
        return "reflux record";
    if (!all_of_parallel(c->h_av.size(), [&](size_t k) {
            const AvgRec &r = c->h_av[k];
            if (!local_ok(c, r.cp, r.cl, true)) return false;
            if (r.fp < 0 || r.fp >= (int)c->patches.size()) return false;
            // the ratio x ratio block of fine cells from fl lies in the
            // interior, as its corners do
            const PatchInfo &F = c->patches[r.fp];
            long long i, j;
            return cell_of(F, r.fl, i, j) && i >= 0 && j >= 0 && i + AMR_RATIO <= F.nx &&
                   j + AMR_RATIO <= F.ny;
        }))
        return "average-down record";
    return nullptr;
}

extern "C" {

const char *hsgn_strerror(int code)
{
    switch (code) {
    case HSGN_OK: return "ok";
    case HSGN_EINVAL: return "invalid argument or call order";
    case HSGN_ENOMEM: return "out of memory";
    case HSGN_ECFL: return "Courant number above cfl_max with a fixed step";
    case HSGN_ENONHYP: return "system not hyperbolic (g h + p + c^2 <= 0)";
    case HSGN_ENAN: return "non-finite value";
    case HSGN_ERANGE: return "gauge outside the scenario's patches";
    case HSGN_EDEVICE: return "HIP runtime error";
    case HSGN_ENOTSUP: return "not supported";
    case HSGN_ESCRATCH: return "grid larger than the static working memory of hsgn_advance_static";
    default: return "unknown status";
    }
}

const char *hsgn_last_error(hsgn_ctx *c) { return c ? c->last_error.c_str() : ""; }

// parameter checks shared by hsgn_create and hsgn_advance_static
static int check_params(const hsgn_params *p)
{
    if ((p->model != 0 && p->model != 1) || (p->precision != 0 && p->precision != 1))
        return HSGN_ENOTSUP;
    if (!(p->g > 0) || p->alpha < 0 || !(p->dry_tol >= 0) || !(p->cfl > 0) ||
        !(p->cfl_max >= p->cfl) || p->nbr_n < 0 || p->nbr_n > 2 || p->limiter < 0 ||
        p->limiter > 3 || (p->transverse != 0 && p->transverse != 2) ||
        (p->splitting != 0 && p->splitting != 1) || !(p->xi1 > 0) || !(p->c2 >= 0))
        return HSGN_EINVAL;
    return HSGN_OK;
}

static StepParams step_params(const hsgn_params *p)
{
    StepParams P;
    P.g = p->g;
    P.a2g = p->c2 > 0.0 ? 0.0 : p->alpha * p->alpha * p->g;
    P.c2f = p->c2 > 0.0 ? p->c2 : 0.0;
    P.eta0 = p->eta0; P.h_star = p->h_star; P.dry_tol = p->dry_tol;
    P.xi0 = p->xi0; P.xi1 = p->xi1; P.kappa = p->kappa;
    P.limiter = p->limiter; P.transverse = p->transverse; P.splitting = p->splitting;
    P.model = p->model;
    return P;
}

int hsgn_create(const hsgn_params *p, void *hip_stream, hsgn_ctx **out)
{
    if (!p || !out) return HSGN_EINVAL;
    *out = nullptr;
    int prc = check_params(p);
    if (prc) return prc;
    hsgn_ctx *c = new (std::nothrow) hsgn_ctx();
    if (!c) return HSGN_ENOMEM;
    c->prm = *p;
    c->mixed = p->precision == 1;
    // HSGN_NO_KERNEL_SPLIT=1 keeps every mixed item on the full kernel (a
    // diagnostic: results are the same bit for bit)
    const char *nosplit = getenv("HSGN_NO_KERNEL_SPLIT");
    c->split = c->mixed && !(nosplit && nosplit[0] == '1');
    // HSGN_NO_PACKING=1 gives every strip of a patch set its own wavefront (a
    // diagnostic: the state is the same bit for bit)
    const char *nopack = getenv("HSGN_NO_PACKING");
    c->pack = !(nopack && nopack[0] == '1');
    c->stream = (hipStream_t)hip_stream;
    c->P = step_params(p);
    *out = c;
    return HSGN_OK;
}

int hsgn_add_grid(hsgn_ctx *c, int scenario, int level, int nx, int ny, double x0, double y0,
                  double dx, double dy, const int bc[4], int *patch_id)
{
    if (!c) return HSGN_EINVAL;
    if (c->finalized) return fail(c, HSGN_EINVAL, "add_grid after finalize");
    if (scenario < 0 || level < 0 || level > 5 || nx < 4 || ny < 4 || !(dx > 0) || !(dy > 0) ||
        !bc)
        return fail(c, HSGN_EINVAL, "bad grid arguments");
    for (int k = 0; k < 4; k++)
        if (bc[k] < 0 || bc[k] > 2) return fail(c, HSGN_EINVAL, "bad boundary condition");
    if ((bc[0] == HSGN_BC_PERIODIC) != (bc[1] == HSGN_BC_PERIODIC) ||
        (bc[2] == HSGN_BC_PERIODIC) != (bc[3] == HSGN_BC_PERIODIC))
        return fail(c, HSGN_EINVAL, "periodic sides must come in pairs");
    if ((long long)(nx + 4) * (ny + 4) > (1LL << 30)) return fail(c, HSGN_EINVAL, "patch too large");
    if ((int)c->scen.size() <= scenario) c->scen.resize(scenario + 1);
    PatchInfo pi;
    memset(&pi, 0, sizeof(pi));
    pi.nx = nx; pi.ny = ny; pi.pitch = nx; pi.scen = scenario;
    for (int k = 0; k < 4; k++) pi.bc[k] = bc[k];
    pi.dx = dx; pi.dy = dy;
    pi.level = level;
    pi.eoff = -1;
    c->patches.push_back(pi);
    c->px0.push_back(x0);
    c->py0.push_back(y0);
    c->pI0.push_back(0);
    c->pJ0.push_back(0);
    int id = (int)c->patches.size() - 1;
    c->scen[scenario].patches.push_back(id);
    if (patch_id) *patch_id = id;
    return HSGN_OK;
}

// rows per marching tile for the patches of one refinement level.  A tile
// of th rows costs th + 4 row iterations (2 halo rows below and above) and
// the chip runs 256 CUs x 4 SIMDs x (2 wavefronts in mixed precision, 1 in
// FP64) tiles at a time, so a level of W(th) tiles takes about
// ceil(W(th) / slots) * (th + 4) row times; the smallest such cost wins
// (ties: the taller tile).
static int model_rows(const hsgn_ctx *c, int level)
{
    const long long slots = 256LL * 4 * (c->mixed ? 2 : 1);
    int best = 64;
    long long best_cost = -1;
    for (int th = 64; th >= 2; th--) {
        long long waves = 0;
        for (const PatchInfo &p : c->patches)
            if (p.level == level) waves += (long long)((p.nx + 59) / 60) * ((p.ny + th - 1) / th);
        long long cost = ((waves + slots - 1) / slots) * (th + 4);
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = th; }
    }
    return best;
}

static int choose_rows(const hsgn_ctx *c, int level)
{
    return c->prm.tile_rows > 0 ? c->prm.tile_rows : model_rows(c, level);
}

// marching work items with tile heights th[level]: clock slots in order; on
// level 0 the single grids come before the patch sets (they use different
// kernel instantiations); fills each slot's work range and each level's
// ranges
// narrow strips of one clock slot packed into items of 64 lanes (2 + w + 2
// each, at most PACK_SEGS per item): best fit decreasing, per tile height.
// The strips are sorted by tile height and width (descending, stable) and
// each goes to the open item with the least room that holds it (the last
// opened of those), else to a new one.  An item left with one strip stays a
// plain item.
struct PackUnit {
    int pid, i0, r0, th, lanes;
};

static void pack_units(std::vector<PackUnit> &u, std::vector<WorkItem> &work,
                       std::vector<PackedItem> &packs)
{
    std::stable_sort(u.begin(), u.end(), [](const PackUnit &a, const PackUnit &b) {
        return a.th != b.th ? a.th > b.th : a.lanes > b.lanes;
    });
    size_t i = 0;
    while (i < u.size()) {
        size_t j = i;
        while (j < u.size() && u[j].th == u[i].th) j++;
        std::vector<PackedItem> bins;
        std::vector<int> used;
        std::vector<std::vector<int>> byroom(65);     // open items by lanes left
        for (size_t k = i; k < j; k++) {
            const int L = u[k].lanes;
            int b = -1;
            for (int r = L; r <= 64 && b < 0; r++)
                if (!byroom[r].empty()) {
                    b = byroom[r].back();
                    byroom[r].pop_back();
                }
            if (b < 0) {
                b = (int)bins.size();
                bins.push_back(PackedItem{});
                used.push_back(0);
            }
            PackedItem &pk = bins[b];
            const int g = pk.nseg++;
            pk.patch[g] = u[k].pid; pk.i0[g] = u[k].i0; pk.r0[g] = u[k].r0; pk.th[g] = u[k].th;
            pk.l0[g] = used[b];
            used[b] += L;
            if (pk.nseg < PACK_SEGS && 64 - used[b] >= 5) byroom[64 - used[b]].push_back(b);
        }
        for (const PackedItem &pk : bins) {
            if (pk.nseg == 1) {
                work.push_back({pk.patch[0], pk.i0[0], pk.r0[0], pk.th[0]});
            } else {
                packs.push_back(pk);
                work.push_back({-1 - (int)(packs.size() - 1), 0, 0, pk.th[0]});
            }
        }
        i = j;
    }
}

// every packed item: 2..PACK_SEGS strips of patch-set patches of one clock
// slot, each narrower than 60 columns and inside its patch, laid on
// consecutive lanes within the 64, its tile height the item's (checked on
// the host before the table reaches the device)
static bool packs_ok(const hsgn_ctx *c, const std::vector<WorkItem> &work,
                     const std::vector<PackedItem> &packs)
{
    if (!packs.empty() && c->mixed && c->mapped_amr) return false;
    std::vector<char> seen(packs.size(), 0);
    for (const WorkItem &w : work) {
        if (w.patch >= 0) continue;
        const long long q = -1LL - w.patch;
        if (q >= (long long)packs.size() || seen[(size_t)q]) return false;
        seen[(size_t)q] = 1;
        const PackedItem &pk = packs[(size_t)q];
        if (pk.nseg < 2 || pk.nseg > PACK_SEGS) return false;
        int lane = 0, slot = -1;
        for (int g = 0; g < pk.nseg; g++) {
            if (pk.patch[g] < 0 || pk.patch[g] >= (int)c->patches.size()) return false;
            const PatchInfo &p = c->patches[pk.patch[g]];
            if (p.frame == 0 || (slot >= 0 && p.scen != slot)) return false;
            slot = p.scen;
            const int wdt = p.nx - pk.i0[g];
            if (pk.i0[g] < 0 || wdt < 1 || wdt >= 60) return false;
            if (pk.r0[g] < 0 || pk.th[g] != w.th || pk.r0[g] + pk.th[g] > p.ny) return false;
            if (pk.l0[g] != lane) return false;
            lane += wdt + 4;
        }
        if (lane > 64) return false;
    }
    for (char x : seen)
        if (!x) return false;
    return true;
}

static void build_work(const hsgn_ctx *c, const std::vector<int> &th, std::vector<WorkItem> &work,
                       std::vector<PackedItem> &packs, std::vector<ScenStatic> &sstat,
                       std::vector<LevelRange> &L)
{
    const int nscen = (int)c->scen.size();
    work.clear();
    packs.clear();
    sstat.assign(c->nslot, ScenStatic());
    auto add_slot_work = [&](int slot) {
        int s = c->slot_scen[slot], l = c->slot_level[slot];
        ScenStatic &ss = sstat[slot];
        const PatchInfo &p0 = c->patches[c->scen[s].lev[l][0]];
        ss.dx = p0.dx;
        ss.dy = p0.dy;
        ss.cfl = c->prm.cfl;
        ss.cfl_max = c->prm.cfl_max;
        ss.w0 = (int)work.size();
        const int t = th[l];
        // patch sets: strips narrower than 60 columns are packed (below),
        // except on mapped patch sets in mixed precision, whose kernel
        // without the FP64 edge solve keeps the patch data uniform (read per
        // lane, it would not fit in its registers)
        const bool packable = c->pack && c->scen[s].amr && !(c->mixed && c->mapped_amr);
        std::vector<PackUnit> units;
        for (int pid : c->scen[s].lev[l]) {
            const PatchInfo &p = c->patches[pid];
            for (int r0 = 0; r0 < p.ny; r0 += t)
                for (int i0 = 0; i0 < p.nx; i0 += 60) {
                    const int h = std::min(t, p.ny - r0), w = std::min(60, p.nx - i0);
                    if (packable && w < 60) units.push_back({pid, i0, r0, h, w + 4});
                    else work.push_back({pid, i0, r0, h});
                }
        }
        if (!units.empty()) pack_units(units, work, packs);
        ss.w1 = (int)work.size();
    };
    L[0].w0 = 0;
    L[0].s0 = 0;
    L[0].s1 = nscen;
    for (int s = 0; s < nscen; s++)
        if (!c->scen[s].amr) add_slot_work(s);
    L[0].wa = (int)work.size();
    for (int s = 0; s < nscen; s++)
        if (c->scen[s].amr) add_slot_work(s);
    L[0].w1 = (int)work.size();
    for (int l = 1; l < c->nlev; l++) {
        L[l].w0 = L[l].wa = (int)work.size();
        L[l].s0 = -1;
        for (int slot = nscen; slot < c->nslot; slot++)
            if (c->slot_level[slot] == l) {
                if (L[l].s0 < 0) L[l].s0 = slot;
                L[l].s1 = slot + 1;
                add_slot_work(slot);
            }
        L[l].w1 = (int)work.size();
    }
}

// a new work table (tile heights th) in place of the context's: device
// buffers grown where it is larger, uploaded, the split's bottom classes
// marked for recomputation and a captured step graph dropped
static int install_work(hsgn_ctx *c, const std::vector<int> &th)
{
    std::vector<WorkItem> work;
    std::vector<PackedItem> packs;
    std::vector<ScenStatic> sstat;
    std::vector<LevelRange> L2 = c->L;
    build_work(c, th, work, packs, sstat, L2);
    if (!packs_ok(c, work, packs)) return fail(c, HSGN_EINVAL, "internal table check: packed items");
    if (packs.size() > c->packs.size()) {
        PackedItem *np = nullptr;
        HIPCHK(c, hipMalloc(&np, sizeof(PackedItem) * packs.size()));
        (void)hipFree(c->d_packs);
        c->d_packs = np;
    }
    if (!packs.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_packs, packs.data(), sizeof(PackedItem) * packs.size(),
                                 hipMemcpyHostToDevice, c->stream));
    if (work.size() > c->work.size()) {
        WorkItem *nw = nullptr;
        double *nc = nullptr;
        int *nlist = nullptr, *nclsb = nullptr, *ncls = nullptr;
        HIPCHK(c, hipMalloc(&nw, sizeof(WorkItem) * work.size()));
        HIPCHK(c, hipMalloc(&nc, sizeof(double) * work.size()));
        HIPCHK(c, hipMalloc(&nlist, sizeof(int) * 2 * work.size()));
        HIPCHK(c, hipMalloc(&ncls, sizeof(int) * work.size()));
        HIPCHK(c, hipMalloc(&nclsb, sizeof(int) * work.size()));
        (void)hipFree(c->d_work);
        (void)hipFree(c->clip);
        (void)hipFree(c->d_list);
        (void)hipFree(c->d_cls);
        (void)hipFree(c->d_clsb);
        c->d_work = nw;
        c->clip = nc;
        c->d_list = nlist;
        c->d_cls = ncls;
        c->d_clsb = nclsb;
    }
    HIPCHK(c, hipMemsetAsync(c->clip, 0, sizeof(double) * work.size(), c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_work, work.data(), sizeof(WorkItem) * work.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_sstat, sstat.data(), sizeof(ScenStatic) * sstat.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->work = work;
    c->packs = packs;
    c->sstat = sstat;
    c->L = L2;
    c->th_level = th;
    c->clsb_dirty = true;
    drop_graph(c);
    return HSGN_OK;
}

// geometry checks of the scenarios and level structure
static int check_scenarios(hsgn_ctx *c)
{
    c->nlev = 1;
    c->any_amr = false;
    for (size_t s = 0; s < c->scen.size(); s++) {
        ScenHost &sh = c->scen[s];
        if (sh.patches.empty()) return fail(c, HSGN_EINVAL, "scenario numbers must be dense");
        sh.amr = sh.patches.size() > 1;
        int nl = 0;
        for (int pid : sh.patches) nl = std::max(nl, c->patches[pid].level + 1);
        sh.lev.assign(nl, std::vector<int>());
        for (int pid : sh.patches) sh.lev[c->patches[pid].level].push_back(pid);
        for (int l = 0; l < nl; l++)
            if (sh.lev[l].empty()) return fail(c, HSGN_EINVAL, "refinement levels must be dense");
        if (!sh.amr) continue;
        c->any_amr = true;
        c->nlev = std::max(c->nlev, nl);
        const PatchInfo &f = c->patches[sh.lev[0][0]];
        double dx0 = f.dx, dy0 = f.dy;
        for (int k = 0; k < 4; k++) sh.bc[k] = f.bc[k];
        sh.X0 = 1e300; sh.Y0 = 1e300;
        for (int pid : sh.lev[0]) {
            const PatchInfo &p = c->patches[pid];
            if (p.dx != dx0 || p.dy != dy0) return fail(c, HSGN_EINVAL, "level-0 patches share dx, dy");
            for (int k = 0; k < 4; k++)
                if (p.bc[k] != sh.bc[k])
                    return fail(c, HSGN_EINVAL, "level-0 patches share the domain boundary conditions");
            sh.X0 = std::min(sh.X0, c->px0[pid]);
            sh.Y0 = std::min(sh.Y0, c->py0[pid]);
        }
        sh.NX = 0; sh.NY = 0;
        for (int pid : sh.patches) {
            PatchInfo &p = c->patches[pid];
            double r = std::pow((double)AMR_RATIO, p.level);
            if (std::fabs(p.dx * r - dx0) > 1e-9 * dx0 || std::fabs(p.dy * r - dy0) > 1e-9 * dy0)
                return fail(c, HSGN_EINVAL, "level-l spacing must be the level-0 spacing / 4^l");
            double ux = p.level ? p.dx * AMR_RATIO : p.dx, uy = p.level ? p.dy * AMR_RATIO : p.dy;
            double ax = (c->px0[pid] - sh.X0) / ux, ay = (c->py0[pid] - sh.Y0) / uy;
            if (std::fabs(ax - std::round(ax)) > 1e-6 || std::fabs(ay - std::round(ay)) > 1e-6)
                return fail(c, HSGN_EINVAL, "patch corner not aligned to the coarser level's cells");
            if (p.level && (p.nx % AMR_RATIO || p.ny % AMR_RATIO))
                return fail(c, HSGN_EINVAL, "refined patch sides must be multiples of 4");
            long long k = p.level ? AMR_RATIO : 1;
            c->pI0[pid] = (int)(std::llround(ax) * k);
            c->pJ0[pid] = (int)(std::llround(ay) * k);
            if (p.level == 0) {
                sh.NX = std::max(sh.NX, c->pI0[pid] + p.nx);
                sh.NY = std::max(sh.NY, c->pJ0[pid] + p.ny);
            }
        }
        for (int pid : sh.lev[0])
            if (c->pI0[pid] < 0 || c->pJ0[pid] < 0) return fail(c, HSGN_EINVAL, "bad level-0 layout");
    }
    return HSGN_OK;
}

}  // extern "C"

// a host table into its device buffer (on the context's stream)
template <class T, class A>
static int upload(hsgn_ctx *c, T *d, const std::vector<T, A> &h)
{
    if (h.empty()) return HSGN_OK;
    HIPCHK(c, hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, c->stream));
    return HSGN_OK;
}

extern "C" {

int hsgn_finalize(hsgn_ctx *c)
{
    if (!c) return HSGN_EINVAL;
    if (c->finalized) return fail(c, HSGN_EINVAL, "finalize called twice");
    if (c->patches.empty()) return fail(c, HSGN_EINVAL, "no patches");
    int rc = check_scenarios(c);
    if (rc) return rc;
    const int nscen = (int)c->scen.size();
    // storage: patch sets keep a 2-cell ghost frame
    long long qo = 0, co = 0;
    for (size_t s = 0; s < c->scen.size(); s++)
        for (int pid : c->scen[s].patches) {
            PatchInfo &p = c->patches[pid];
            p.frame = c->scen[s].amr ? 2 : 0;
            p.pitch = p.nx + 2 * p.frame;
            p.plane = (long long)p.pitch * (p.ny + 2 * p.frame);
            long long org = (long long)p.frame * p.pitch + p.frame;
            p.qoff = qo + org;
            p.coff = co + org;
            qo += 7 * p.plane;
            co += p.plane;
        }
    c->qtotal = qo;
    c->ctotal = co;
    // clock slots: scenario s is slot s (its level 0); finer levels of patch
    // sets follow, level by level
    c->nslot = nscen;
    std::vector<int> slot_level(nscen, 0), slot_scen(nscen);
    for (int s = 0; s < nscen; s++) {
        c->scen[s].slot.assign(c->scen[s].lev.size(), -1);
        c->scen[s].slot[0] = s;
        slot_scen[s] = s;
    }
    for (int l = 1; l < c->nlev; l++)
        for (int s = 0; s < nscen; s++)
            if ((int)c->scen[s].lev.size() > l) {
                c->scen[s].slot[l] = c->nslot++;
                slot_level.push_back(l);
                slot_scen.push_back(s);
            }
    for (int s = 0; s < nscen; s++)
        for (size_t l = 0; l < c->scen[s].lev.size(); l++)
            for (int pid : c->scen[s].lev[l]) c->patches[pid].scen = c->scen[s].slot[l];
    // boundary-flux entries of refined patches, level by level
    c->L.assign(c->nlev, LevelRange());
    c->etotal = 0;
    for (int l = 1; l < c->nlev; l++) {
        c->L[l].e0 = c->etotal;
        for (int s = 0; s < nscen; s++)
            if ((int)c->scen[s].lev.size() > l)
                for (int pid : c->scen[s].lev[l]) {
                    PatchInfo &p = c->patches[pid];
                    p.eoff = c->etotal;
                    c->etotal += 2LL * (p.nx + p.ny);
                }
        c->L[l].e1 = c->etotal;
    }
    c->slot_scen = slot_scen;
    c->slot_level = slot_level;
    c->th_level.assign(c->nlev, 0);
    for (int l = 0; l < c->nlev; l++) c->th_level[l] = choose_rows(c, l);
    build_work(c, c->th_level, c->work, c->packs, c->sstat, c->L);
    if (!packs_ok(c, c->work, c->packs))
        return fail(c, HSGN_EINVAL, "internal table check: packed items");
    // patch-set tables, grouped by level
    {
        std::vector<std::vector<PatchRecs>> recs(c->nlev);
        std::vector<std::vector<RefluxRec>> lrf(c->nlev);
        for (int s = 0; s < nscen; s++)
            if (c->scen[s].amr && (rc = build_patch_set(c, s, recs, lrf))) return rc;
        // the tables grouped by level (scenarios, then patches, in order):
        // offsets first, then the records copied into place on host threads
        struct Off { size_t gc, gi, fr, av; };
        std::vector<std::vector<Off>> off(c->nlev);
        size_t ngc = 0, ngi = 0, nfr = 0, nav = 0, nrf = 0;
        for (int l = 0; l < c->nlev; l++) {
            LevelRange &R = c->L[l];
            R.gc0 = (int)ngc; R.gi0 = (int)ngi; R.fr0 = (int)nfr; R.av0 = (int)nav;
            for (const PatchRecs &r : recs[l]) {
                off[l].push_back({ngc, ngi, nfr, nav});
                ngc += r.gc.size(); ngi += r.gi.size(); nfr += r.fr.size(); nav += r.av.size();
            }
            R.gc1 = (int)ngc; R.gi1 = (int)ngi; R.fr1 = (int)nfr; R.av1 = (int)nav;
            R.rf0 = (int)nrf;
            nrf += lrf[l].size();
            R.rf1 = (int)nrf;
        }
        // sized without zeroing; memory lent by the context this one replaces
        // is reused, a table that outgrows it gets a quarter to spare
        auto size_table = [](auto &v, size_t n) {
            v.clear();
            if (v.capacity() < n) v.reserve(n + n / 4);
            v.resize(n);
        };
        size_table(c->h_gc, ngc);
        size_table(c->h_gi, ngi);
        size_table(c->h_fr, nfr);
        size_table(c->h_av, nav);
        c->ngc = (int)ngc;
        c->ngi = (int)ngi;
        c->h_rf.clear();
        c->h_rf.reserve(nrf);
        for (int l = 0; l < c->nlev; l++) c->h_rf.insert(c->h_rf.end(), lrf[l].begin(), lrf[l].end());
        std::vector<std::pair<int, int>> jobs;         // (level, patch entry)
        for (int l = 0; l < c->nlev; l++)
            for (size_t k = 0; k < recs[l].size(); k++) jobs.push_back({l, (int)k});
        auto place = [&](int t, int nt) {
            for (size_t j = (size_t)t; j < jobs.size(); j += (size_t)nt) {
                PatchRecs &r = recs[jobs[j].first][jobs[j].second];
                const Off &o = off[jobs[j].first][jobs[j].second];
                std::copy(r.gc.begin(), r.gc.end(), c->h_gc.begin() + o.gc);
                std::copy(r.gi.begin(), r.gi.end(), c->h_gi.begin() + o.gi);
                std::copy(r.fr.begin(), r.fr.end(), c->h_fr.begin() + o.fr);
                std::copy(r.av.begin(), r.av.end(), c->h_av.begin() + o.av);
                // released here, on the workers, rather than one by one after
                std::vector<GhostCopy>().swap(r.gc);
                std::vector<GhostInterp>().swap(r.gi);
                std::vector<FluxRec>().swap(r.fr);
                std::vector<AvgRec>().swap(r.av);
            }
        };
        const int nt = jobs.size() > 64 ? 4 * host_threads() : 1;
        HostPool::get().parallel_for(nt, [&](int t) { place(t, nt); });
    }
    // the tables are checked on a host thread while the device buffers are
    // allocated and the tables uploaded: no kernel reads them before the
    // check has passed, and a failed check leaves the context unfinalized
    const char *table_bad = nullptr;
    std::thread checker([&]() { table_bad = table_error(c); });
    struct JoinAtExit {
        std::thread &t;
        ~JoinAtExit() { if (t.joinable()) t.join(); }
    } join_checker{checker};
    // the buffers fixed here share one device allocation, freed at once with
    // the context; the work-table buffers (which the tile-height tuner
    // replaces) and the gauge buffers are allocated on their own
    long long big = 0;
    for (const PatchInfo &p : c->patches) big = std::max<long long>(big, 7LL * p.nx * p.ny);
    c->stage_len = big;
    char *base = nullptr;
    size_t off = 0;
    auto carve = [&](auto *&ptr, size_t n) {
        using T = std::remove_reference_t<decltype(*ptr)>;
        const size_t bytes = sizeof(T) * n;
        ptr = base && bytes ? reinterpret_cast<T *>(base + off) : nullptr;
        off += (bytes + 255) / 256 * 256;
    };
    auto carve_all = [&]() {
        off = 0;
        if (c->mixed) {
            carve(c->f0, (size_t)c->qtotal);
            carve(c->f1, (size_t)c->qtotal);
            carve(c->fbath, (size_t)c->ctotal);
        } else {
            carve(c->q0, (size_t)c->qtotal);
            carve(c->q1, (size_t)c->qtotal);
            carve(c->bath, (size_t)c->ctotal);
        }
        carve(c->stage, (size_t)big);
        carve(c->m0, (size_t)c->ctotal);
        carve(c->m1, (size_t)c->ctotal);
        carve(c->d_patches, c->patches.size());
        carve(c->d_keep, c->patches.size());
        carve(c->d_lcnt, 2);
        // the classes of a context of single grids change within an advance
        // only where a cell latches (patch sets also take masks from other
        // levels' and patches' cells into their ghost frames: they classify
        // every attempt)
        carve(c->d_latch, c->split && !c->any_amr ? 1 : 0);
        carve(c->d_scen, (size_t)c->nslot);
        carve(c->d_sstat, (size_t)c->nslot);
        carve(c->d_slots, (size_t)c->nslot);
        carve(c->d_cnt, 2);
        carve(c->d_err, 1);
        carve(c->d_mass, 2);
        carve(c->d_E, 7 * (size_t)c->etotal);
        carve(c->d_R, 7 * (size_t)c->etotal);
        carve(c->d_rclip, c->h_rf.size());
        carve(c->d_gc, c->h_gc.size());
        carve(c->d_gi, c->h_gi.size());
        carve(c->d_fr, c->h_fr.size());
        carve(c->d_rf, c->h_rf.size());
        carve(c->d_av, c->h_av.size());
    };
    carve_all();                                  // sizes
    HIPCHK(c, hipMalloc(&c->arena, std::max<size_t>(off, 256)));
    base = static_cast<char *>(c->arena);
    carve_all();                                  // addresses
    const size_t sq = c->mixed ? sizeof(float) : sizeof(double);
    HIPCHK(c, hipMemsetAsync(c->mixed ? (void *)c->f0 : (void *)c->q0, 0, sq * c->qtotal, c->stream));
    HIPCHK(c, hipMemsetAsync(c->mixed ? (void *)c->f1 : (void *)c->q1, 0, sq * c->qtotal, c->stream));
    HIPCHK(c, hipMemsetAsync(c->mixed ? (void *)c->fbath : (void *)c->bath, 0, sq * c->ctotal,
                             c->stream));
    HIPCHK(c, hipMemsetAsync(c->m0, 0, c->ctotal, c->stream));
    HIPCHK(c, hipMemsetAsync(c->m1, 0, c->ctotal, c->stream));
    if (c->etotal > 0) {
        HIPCHK(c, hipMemsetAsync(c->d_E, 0, sizeof(double) * 7 * c->etotal, c->stream));
        HIPCHK(c, hipMemsetAsync(c->d_R, 0, sizeof(double) * 7 * c->etotal, c->stream));
    }
    if (!c->h_rf.empty())
        HIPCHK(c, hipMemsetAsync(c->d_rclip, 0, sizeof(double) * c->h_rf.size(), c->stream));
    c->state_set.assign(c->patches.size(), 0);
    HIPCHK(c, hipMalloc(&c->clip, sizeof(double) * std::max<size_t>(c->work.size(), 1)));
    HIPCHK(c, hipMalloc(&c->d_work, sizeof(WorkItem) * c->work.size()));
    HIPCHK(c, hipMalloc(&c->d_packs, sizeof(PackedItem) * std::max<size_t>(c->packs.size(), 1)));
    HIPCHK(c, hipMalloc(&c->d_list, sizeof(int) * 2 * std::max<size_t>(c->work.size(), 1)));
    HIPCHK(c, hipMalloc(&c->d_cls, sizeof(int) * std::max<size_t>(c->work.size(), 1)));
    HIPCHK(c, hipMalloc(&c->d_clsb, sizeof(int) * std::max<size_t>(c->work.size(), 1)));
    HIPCHK(c, hipMemsetAsync(c->clip, 0, sizeof(double) * std::max<size_t>(c->work.size(), 1),
                             c->stream));
    c->clsb_dirty = true;
    if (c->split) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    if ((rc = upload(c, c->d_gc, c->h_gc)) || (rc = upload(c, c->d_gi, c->h_gi)) ||
        (rc = upload(c, c->d_fr, c->h_fr)) || (rc = upload(c, c->d_rf, c->h_rf)) ||
        (rc = upload(c, c->d_av, c->h_av)))
        return rc;
    HIPCHK(c, hipMemcpyAsync(c->d_patches, c->patches.data(), sizeof(PatchInfo) * c->patches.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_work, c->work.data(), sizeof(WorkItem) * c->work.size(),
                             hipMemcpyHostToDevice, c->stream));
    if (!c->packs.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_packs, c->packs.data(), sizeof(PackedItem) * c->packs.size(),
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_sstat, c->sstat.data(), sizeof(ScenStatic) * c->nslot,
                             hipMemcpyHostToDevice, c->stream));
    std::vector<ScenState> st(c->nslot);
    memset(st.data(), 0, sizeof(ScenState) * c->nslot);
    HIPCHK(c, hipMemcpyAsync(c->d_scen, st.data(), sizeof(ScenState) * c->nslot,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    checker.join();
    if (table_bad) return fail(c, HSGN_EINVAL, std::string("internal table check: ") + table_bad);
    c->finalized = true;
    c->amr_dirty = c->any_amr;
    return HSGN_OK;
}

// the split step's latch flag set (every lane of one wavefront stores it,
// a vector store)
__global__ void set_flag_kernel(int *flag, int v)
{
    if (threadIdx.x < 64) *flag = v;
}

static int pull_scen(hsgn_ctx *c, std::vector<ScenState> &st)
{
    st.resize(c->nslot);
    HIPCHK(c, hipMemcpyAsync(st.data(), c->d_scen, sizeof(ScenState) * st.size(),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

static int push_scen(hsgn_ctx *c, const std::vector<ScenState> &st)
{
    HIPCHK(c, hipMemcpyAsync(c->d_scen, st.data(), sizeof(ScenState) * st.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

static int check_patch(hsgn_ctx *c, int patch)
{
    if (!c) return HSGN_EINVAL;
    if (!c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (patch < 0 || patch >= (int)c->patches.size()) return fail(c, HSGN_EINVAL, "bad patch id");
    return HSGN_OK;
}

static hipMemcpyKind kind_in(int on_device)
{
    return on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
static hipMemcpyKind kind_out(int on_device)
{
    return on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

static unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

// patch sets: coarse bathymetry under refined patches (mean of the fine one,
// finest level first), ghost bathymetry, phi_T and the interface flags
static int ensure_prepared(hsgn_ctx *c)
{
    if (!c->any_amr || !c->amr_dirty) return HSGN_OK;
    // a patch set is mapped in every patch or in none
    for (const ScenHost &sh : c->scen) {
        if (!sh.amr) continue;
        size_t nm = 0;
        for (int pid : sh.patches) nm += c->patches[pid].metric ? 1 : 0;
        if (nm != 0 && nm != sh.patches.size())
            return fail(c, HSGN_EINVAL, "a patch set is mapped in every patch or in none");
    }
    if (c->mixed)
        HIPCHK(c, hipMemcpy(c->d_keep, c->state_set.data(), c->state_set.size(),
                            hipMemcpyHostToDevice));
    for (int l = c->nlev - 1; l >= 1; l--) {
        const LevelRange &R = c->L[l];
        if (c->mixed)
            launch_avgdown32(amr_buffers<float>(c, c->f0, c->f1, c->fbath), c->d_av + R.av0,
                             R.av1 - R.av0, true, c->stream, c->d_keep);
        else
            launch_avgdown64(amr_buffers<double>(c, c->q0, c->q1, c->bath), c->d_av + R.av0,
                             R.av1 - R.av0, true, c->stream);
    }
    const int nc = c->ngc, ni = c->ngi;
    if (c->mixed)
        launch_ghost_bath32(amr_buffers<float>(c, c->f0, c->f1, c->fbath), c->d_gc, nc, c->d_gi, ni,
                            c->stream);
    else
        launch_ghost_bath64(amr_buffers<double>(c, c->q0, c->q1, c->bath), c->d_gc, nc, c->d_gi, ni,
                            c->stream);
    {
        // phi_T of every patch-set patch, one launch (the ghost frames hold
        // the neighbourhood's bathymetry)
        std::vector<BulkRec> recs;
        long long tot = 0;
        for (size_t s = 0; s < c->scen.size(); s++) {
            if (!c->scen[s].amr) continue;
            for (int pid : c->scen[s].patches) {
                recs.push_back({c->patches[pid], tot});
                tot += (long long)c->patches[pid].nx * c->patches[pid].ny;
            }
        }
        if (!recs.empty()) {
            BulkRec *d = nullptr;
            HIPCHK(c, hipMalloc(&d, sizeof(BulkRec) * recs.size()));
            hipError_t e = hipMemcpy(d, recs.data(), sizeof(BulkRec) * recs.size(),
                                     hipMemcpyHostToDevice);
            if (e == hipSuccess) {
                if (c->mixed)
                    mask_bulk_kernel<float><<<nblk(tot), 256, 0, c->stream>>>(
                        d, (int)recs.size(), tot, c->fbath, c->m0, c->m1, c->prm.eta0, c->prm.h_star,
                        c->prm.nbr_n);
                else
                    mask_bulk_kernel<double><<<nblk(tot), 256, 0, c->stream>>>(
                        d, (int)recs.size(), tot, c->bath, c->m0, c->m1, c->prm.eta0, c->prm.h_star,
                        c->prm.nbr_n);
                e = hipGetLastError();
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            }
            (void)hipFree(d);
            if (e != hipSuccess)
                return fail(c, HSGN_EDEVICE, std::string("phi_T: ") + hipGetErrorString(e));
        }
    }
    launch_iface(c->d_patches, c->d_rf, (int)c->h_rf.size(), c->m0, c->m1, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->amr_dirty = false;
    return HSGN_OK;
}

// the sponge of scenario s into its patches' PatchInfo (host and device)
static int apply_sponge(hsgn_ctx *c, int s)
{
    const ScenHost &sh = c->scen[s];
    for (int pid : sh.patches) {
        PatchInfo &p = c->patches[pid];
        for (int e = 0; e < 4; e++) p.sp_w[e] = sh.sp_w[e];
        p.sp_rate = sh.sp_rate;
        if (sh.amr) {
            long long f = 1;
            for (int k = 0; k < p.level; k++) f *= AMR_RATIO;
            p.sp_i0 = c->pI0[pid]; p.sp_j0 = c->pJ0[pid];
            p.sp_nx = (long long)sh.NX * f; p.sp_ny = (long long)sh.NY * f;
        } else {
            p.sp_i0 = 0; p.sp_j0 = 0;
            p.sp_nx = p.nx; p.sp_ny = p.ny;
        }
    }
    HIPCHK(c, hipMemcpy(c->d_patches, c->patches.data(), sizeof(PatchInfo) * c->patches.size(),
                        hipMemcpyHostToDevice));
    return HSGN_OK;
}

// metric planes of a mapped patch from its node coordinates [ny + 5][nx + 5]
// (nodes i = -2..nx+2, j = -2..ny+2): per cell of the frame (two ghost
// layers) the capacity (area over dx dy), the unit normal towards
// increasing i and the length ratio (over dy) of its left edge, the same
// towards increasing j (length over dx) for its bottom edge.  False for a
// cell of non-positive area or an edge of zero length.
static bool mapping_metric(const PatchInfo &p, const double *xn, const double *yn,
                           std::vector<double> &out)
{
#pragma clang fp contract(off)
    const long long W = p.nx + 4, MP = W * (p.ny + 4), NW = p.nx + 5;
    out.assign((size_t)(7 * MP), 0.0);
    auto X = [&](int i, int j) { return xn[(long long)(j + 2) * NW + (i + 2)]; };
    auto Y = [&](int i, int j) { return yn[(long long)(j + 2) * NW + (i + 2)]; };
    for (int j = -2; j < p.ny + 2; j++) {
        for (int i = -2; i < p.nx + 2; i++) {
            const long long k = (long long)(j + 2) * W + (i + 2);
            const double area = 0.5 * ((X(i + 1, j + 1) - X(i, j)) * (Y(i, j + 1) - Y(i + 1, j))
                                     - (X(i, j + 1) - X(i + 1, j)) * (Y(i + 1, j + 1) - Y(i, j)));
            const double ex = X(i, j + 1) - X(i, j), ey = Y(i, j + 1) - Y(i, j);
            const double L = std::sqrt(ex * ex + ey * ey);
            const double fx = X(i + 1, j) - X(i, j), fy = Y(i + 1, j) - Y(i, j);
            const double M = std::sqrt(fx * fx + fy * fy);
            if (!(area > 0.0) || !(L > 0.0) || !(M > 0.0) || !std::isfinite(area)) return false;
            out[k] = area / (p.dx * p.dy);
            out[MP + k] = ey / L;
            out[2 * MP + k] = (0.0 - ex) / L;     // +0 for an axis-aligned edge
            out[3 * MP + k] = L / p.dy;
            out[4 * MP + k] = (0.0 - fy) / M;
            out[5 * MP + k] = fx / M;
            out[6 * MP + k] = M / p.dx;
        }
    }
    return true;
}

int hsgn_set_mapping(hsgn_ctx *c, int patch, const double *xn, const double *yn)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!xn || !yn) return fail(c, HSGN_EINVAL, "null node coordinates");
    PatchInfo &p = c->patches[patch];
    if (c->any_sponge) return fail(c, HSGN_ENOTSUP, "mapped grids with a sponge layer");
    std::vector<double> m;
    if (!mapping_metric(p, xn, yn, m))
        return fail(c, HSGN_EINVAL, "mapping with a cell of non-positive area or an edge of zero length");
    // work already queued may still read the patch table and the metric
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->d_metric.size() < c->patches.size()) c->d_metric.resize(c->patches.size(), nullptr);
    if (!c->d_metric[patch])
        HIPCHK(c, hipMalloc((void **)&c->d_metric[patch], sizeof(double) * m.size()));
    HIPCHK(c, hipMemcpy(c->d_metric[patch], m.data(), sizeof(double) * m.size(),
                        hipMemcpyHostToDevice));
    p.metric = c->d_metric[patch];
    // the first mapped patch of a kind switches its step launches to the
    // mapped kernel; a step graph captured before holds the Cartesian one
    bool &kind = p.frame != 0 ? c->mapped_amr : c->mapped_single;
    if (!kind) drop_graph(c);
    kind = true;
    c->any_mapped = true;
    // mixed precision: the mapped patch-set kernels take no packed items
    if (p.frame != 0 && c->mixed && !c->packs.empty()) {
        int rc2 = install_work(c, c->th_level);
        if (rc2) return rc2;
    }
    // a patch set averages its bathymetry down again, weighted by the capacities
    if (p.frame != 0) c->amr_dirty = true;
    HIPCHK(c, hipMemcpy(c->d_patches, c->patches.data(), sizeof(PatchInfo) * c->patches.size(),
                        hipMemcpyHostToDevice));
    return HSGN_OK;
}

int hsgn_set_sponge(hsgn_ctx *c, int scenario, const double width[4], double rate)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (c->any_mapped && rate > 0.0) return fail(c, HSGN_ENOTSUP, "a sponge layer on mapped grids");
    if (scenario < 0 || scenario >= (int)c->scen.size() || c->scen[scenario].patches.empty())
        return fail(c, HSGN_EINVAL, "no such scenario");
    if (!width) return fail(c, HSGN_EINVAL, "null sponge widths");
    if (!(rate >= 0.0) || !std::isfinite(rate)) return fail(c, HSGN_EINVAL, "sponge rate");
    for (int e = 0; e < 4; e++)
        if (!(width[e] >= 0.0) || !std::isfinite(width[e]))
            return fail(c, HSGN_EINVAL, "sponge width");
    ScenHost &sh = c->scen[scenario];
    for (int e = 0; e < 4; e++) sh.sp_w[e] = width[e];
    sh.sp_rate = rate;
    const bool before = c->any_sponge;
    c->any_sponge = false;
    for (const ScenHost &x : c->scen) c->any_sponge = c->any_sponge || x.sp_rate > 0.0;
    if (c->any_sponge != before) drop_graph(c);     // the graph holds the other kernels
    return apply_sponge(c, scenario);
}

int hsgn_set_bathymetry(hsgn_ctx *c, int patch, const double *b, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!b) return fail(c, HSGN_EINVAL, "null bathymetry");
    const PatchInfo &p = c->patches[patch];
    const bool amr = p.frame != 0;       // a patch of a patch set
    long long n = (long long)p.nx * p.ny;
    unsigned nb = nblk(n);
    // host copy of the bathymetry as set: regridding rebuilds from it
    if ((int)c->braw.size() < (int)c->patches.size()) c->braw.resize(c->patches.size());
    if ((int)c->braw_rule.size() < (int)c->patches.size()) c->braw_rule.resize(c->patches.size(), 0);
    c->braw_rule[patch] = 0;
    c->braw[patch].resize((size_t)n);
    c->b0_scen = -1;                      // the cached level-0 bathymetry is stale
    if (on_device)
        HIPCHK(c, hipMemcpy(c->braw[patch].data(), b, sizeof(double) * n, hipMemcpyDeviceToHost));
    else
        memcpy(c->braw[patch].data(), b, sizeof(double) * n);
    if (c->mixed) {
        // stored in FP32; phi_T is computed from the stored values.  A set
        // state keeps its depth under the new bottom (the stored eta' moves
        // with it), as the FP64 storage of h does
        HIPCHK(c, hipMemcpyAsync(c->stage, b, sizeof(double) * n, kind_in(on_device), c->stream));
        if (c->state_set[patch]) {
            std::vector<ScenState> st;
            if ((rc = pull_scen(c, st))) return rc;
            keep_depth_kernel<<<nb, 256, 0, c->stream>>>(p, st[p.scen].cur ? c->f1 : c->f0, c->fbath,
                                                         c->stage, c->prm.eta0);
        }
        scatter_plane_kernel<double, float><<<nb, 256, 0, c->stream>>>(p, c->stage, c->fbath, 0);
        if (!amr)
            mask_kernel<float><<<nb, 256, 0, c->stream>>>(p, c->fbath, c->m0, c->m1, c->prm.eta0,
                                                          c->prm.h_star, c->prm.nbr_n);
    } else {
        if (p.frame) {
            HIPCHK(c, hipMemcpyAsync(c->stage, b, sizeof(double) * n, kind_in(on_device), c->stream));
            scatter_plane_kernel<double, double><<<nb, 256, 0, c->stream>>>(p, c->stage, c->bath, 0);
        } else {
            HIPCHK(c, hipMemcpyAsync(c->bath + p.coff, b, sizeof(double) * n, kind_in(on_device),
                                     c->stream));
        }
        if (!amr)
            mask_kernel<double><<<nb, 256, 0, c->stream>>>(p, c->bath, c->m0, c->m1, c->prm.eta0,
                                                           c->prm.h_star, c->prm.nbr_n);
    }
    if (amr) c->amr_dirty = true;
    c->clsb_dirty = true;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_set_state(hsgn_ctx *c, int patch, const double *q, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!q) return fail(c, HSGN_EINVAL, "null state");
    if ((rc = ensure_prepared(c))) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    const PatchInfo &p = c->patches[patch];
    long long n = (long long)p.nx * p.ny;
    if (c->mixed || p.frame) {
        HIPCHK(c, hipMemcpyAsync(c->stage, q, sizeof(double) * 7 * n, kind_in(on_device), c->stream));
        if (c->mixed)
            to_storage_kernel<float, true><<<nblk(n), 256, 0, c->stream>>>(
                p, c->stage, st[p.scen].cur ? c->f1 : c->f0, c->fbath, c->prm.eta0);
        else
            to_storage_kernel<double, false><<<nblk(n), 256, 0, c->stream>>>(
                p, c->stage, st[p.scen].cur ? c->q1 : c->q0, c->bath, c->prm.eta0);
        HIPCHK(c, hipGetLastError());
    } else {
        double *dst = (st[p.scen].cur ? c->q1 : c->q0) + p.qoff;
        HIPCHK(c, hipMemcpyAsync(dst, q, sizeof(double) * 7 * n, kind_in(on_device), c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->state_set[patch] = 1;
    return HSGN_OK;
}

int hsgn_get_state(hsgn_ctx *c, int patch, double *q, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!q) return fail(c, HSGN_EINVAL, "null output");
    if ((rc = ensure_prepared(c))) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    const PatchInfo &p = c->patches[patch];
    long long n = (long long)p.nx * p.ny;
    if (c->mixed || p.frame) {
        if (c->mixed)
            from_storage_kernel<float, true><<<nblk(n), 256, 0, c->stream>>>(
                p, st[p.scen].cur ? c->f1 : c->f0, c->fbath, c->prm.eta0, c->stage);
        else
            from_storage_kernel<double, false><<<nblk(n), 256, 0, c->stream>>>(
                p, st[p.scen].cur ? c->q1 : c->q0, c->bath, c->prm.eta0, c->stage);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(q, c->stage, sizeof(double) * 7 * n, kind_out(on_device), c->stream));
    } else {
        const double *src = (st[p.scen].cur ? c->q1 : c->q0) + p.qoff;
        HIPCHK(c, hipMemcpyAsync(q, src, sizeof(double) * 7 * n, kind_out(on_device), c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_get_mask(hsgn_ctx *c, int patch, uint8_t *m, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!m) return fail(c, HSGN_EINVAL, "null output");
    if ((rc = ensure_prepared(c))) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    const PatchInfo &p = c->patches[patch];
    long long n = (long long)p.nx * p.ny;
    const uint8_t *src = st[p.scen].cur ? c->m1 : c->m0;
    if (p.frame) {
        uint8_t *tmp = (uint8_t *)c->stage;
        gather_plane_kernel<uint8_t, uint8_t><<<nblk(n), 256, 0, c->stream>>>(p, src, tmp, 1);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(m, tmp, (size_t)n, kind_out(on_device), c->stream));
    } else {
        HIPCHK(c, hipMemcpyAsync(m, src + p.coff, (size_t)n, kind_out(on_device), c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_set_mask(hsgn_ctx *c, int patch, const uint8_t *m, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!m) return fail(c, HSGN_EINVAL, "null mask");
    if ((rc = ensure_prepared(c))) return rc;
    const PatchInfo &p = c->patches[patch];
    long long n = (long long)p.nx * p.ny;
    if (p.frame) {
        uint8_t *tmp = (uint8_t *)c->stage;
        HIPCHK(c, hipMemcpyAsync(tmp, m, (size_t)n, kind_in(on_device), c->stream));
        scatter_plane_kernel<uint8_t, uint8_t><<<nblk(n), 256, 0, c->stream>>>(p, tmp, c->m0, 1);
        scatter_plane_kernel<uint8_t, uint8_t><<<nblk(n), 256, 0, c->stream>>>(p, tmp, c->m1, 1);
        HIPCHK(c, hipGetLastError());
    } else {
        HIPCHK(c, hipMemcpyAsync(c->m0 + p.coff, m, (size_t)n, kind_in(on_device), c->stream));
        HIPCHK(c, hipMemcpyAsync(c->m1 + p.coff, m, (size_t)n, kind_in(on_device), c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

static bool point_in(const hsgn_ctx *c, int pid, double x, double y)
{
    const PatchInfo &p = c->patches[pid];
    return x >= c->px0[pid] && x <= c->px0[pid] + p.nx * p.dx && y >= c->py0[pid] &&
           y <= c->py0[pid] + p.ny * p.dy;
}

// the finest patch of a scenario containing a point (-1: none)
static int finest_patch(const hsgn_ctx *c, int scenario, double x, double y)
{
    const ScenHost &sh = c->scen[scenario];
    for (int l = (int)sh.lev.size() - 1; l >= 0; l--)
        for (int pid : sh.lev[l])
            if (point_in(c, pid, x, y)) return pid;
    return -1;
}

int hsgn_set_gauges(hsgn_ctx *c, int scenario, int n, const double *xy)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (scenario < 0 || scenario >= (int)c->scen.size() || n < 0 || (n > 0 && !xy))
        return fail(c, HSGN_EINVAL, "bad gauge arguments");
    for (int k = 0; k < n; k++)
        if (finest_patch(c, scenario, xy[2 * k], xy[2 * k + 1]) < 0)
            return fail(c, HSGN_ERANGE, "gauge outside the scenario");
    c->scen[scenario].gauge_xy.assign(xy, xy + 2 * n);
    c->scen[scenario].ng = n;
    c->scen[scenario].gcap = 0;     // record area rebuilt on the next advance
    std::vector<ScenState> st;
    int rc = pull_scen(c, st);
    if (rc) return rc;
    st[scenario].records = 0;
    return push_scen(c, st);
}

// (re)build the gauge tables so that every scenario can hold `need` more records
static int ensure_gauges(hsgn_ctx *c, const std::vector<ScenState> &st, long long need)
{
    bool rebuild = false;
    for (size_t s = 0; s < c->scen.size(); s++)
        if (c->scen[s].ng > 0 && st[s].records + need > c->scen[s].gcap) rebuild = true;
    if (!rebuild && (c->d_gauges || c->ngauge_total == 0)) {
        int tot = 0;
        for (auto &s : c->scen) tot += s.ng;
        if (tot == c->ngauge_total) return HSGN_OK;
    }
    drop_graph(c);                  // the step graph holds the old tables
    // keep the records already taken
    std::vector<double> old;
    if (c->rec && c->rec_total > 0) {
        old.resize(c->rec_total);
        HIPCHK(c, hipMemcpyAsync(old.data(), c->rec, sizeof(double) * c->rec_total,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    std::vector<long long> oldoff(c->scen.size()), oldcap(c->scen.size());
    for (size_t s = 0; s < c->scen.size(); s++) { oldoff[s] = c->scen[s].roff; oldcap[s] = c->scen[s].gcap; }
    long long off = 0;
    std::vector<GaugeDev> G;
    for (size_t s = 0; s < c->scen.size(); s++) {
        ScenHost &sh = c->scen[s];
        long long cap = std::max<long long>(st[s].records + need, 2 * sh.gcap);
        if (sh.ng == 0) cap = 0;
        sh.roff = off;
        sh.gcap = cap;
        off += cap * (1 + sh.ng);
        for (int k = 0; k < sh.ng; k++) {
            double x = sh.gauge_xy[2 * k], y = sh.gauge_xy[2 * k + 1];
            int pid = finest_patch(c, (int)s, x, y);
            const PatchInfo &p = c->patches[pid];
            double fx = (x - c->px0[pid]) / p.dx - 0.5;
            double fy = (y - c->py0[pid]) / p.dy - 0.5;
            int i0 = (int)std::floor(fx), j0 = (int)std::floor(fy);
            i0 = std::min(std::max(i0, 0), p.nx - 2);
            j0 = std::min(std::max(j0, 0), p.ny - 2);
            double wx = std::min(std::max(fx - i0, 0.0), 1.0);
            double wy = std::min(std::max(fy - j0, 0.0), 1.0);
            GaugeDev g;
            memset(&g, 0, sizeof(g));
            g.scen = (int)s; g.slot = k; g.ng = sh.ng;
            g.qscen = p.scen;
            g.qoff = p.qoff; g.plane = p.coff;
            g.c00 = (long long)j0 * p.pitch + i0;
            g.c01 = g.c00 + 1;
            g.c10 = g.c00 + p.pitch;
            g.c11 = g.c10 + 1;
            g.wx = wx; g.wy = wy;
            g.roff = sh.roff; g.cap = cap;
            G.push_back(g);
        }
    }
    double *nrec = nullptr;
    if (off > 0) HIPCHK(c, hipMalloc(&nrec, sizeof(double) * off));
    for (size_t s = 0; s < c->scen.size(); s++) {
        long long keep = std::min<long long>(st[s].records, oldcap[s]);
        if (keep > 0 && !old.empty() && c->scen[s].ng > 0)
            HIPCHK(c, hipMemcpyAsync(nrec + c->scen[s].roff, old.data() + oldoff[s],
                                     sizeof(double) * keep * (1 + c->scen[s].ng),
                                     hipMemcpyHostToDevice, c->stream));
    }
    if (c->rec) (void)hipFree(c->rec);
    c->rec = nrec;
    c->rec_total = off;
    if (c->d_gauges) (void)hipFree(c->d_gauges);
    c->d_gauges = nullptr;
    c->ngauge_total = (int)G.size();
    if (!G.empty()) {
        HIPCHK(c, hipMalloc(&c->d_gauges, sizeof(GaugeDev) * G.size()));
        HIPCHK(c, hipMemcpyAsync(c->d_gauges, G.data(), sizeof(GaugeDev) * G.size(),
                                 hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_read_gauges(hsgn_ctx *c, int scenario, double *t, double *eta, int max_records,
                     int *n_records)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (scenario < 0 || scenario >= (int)c->scen.size() || !n_records)
        return fail(c, HSGN_EINVAL, "bad arguments");
    std::vector<ScenState> st;
    int rc = pull_scen(c, st);
    if (rc) return rc;
    ScenHost &sh = c->scen[scenario];
    long long n = std::min<long long>(st[scenario].records, sh.gcap);
    n = std::min<long long>(n, max_records);
    *n_records = (int)n;
    if (n > 0 && sh.ng > 0) {
        std::vector<double> buf(n * (1 + sh.ng));
        HIPCHK(c, hipMemcpyAsync(buf.data(), c->rec + sh.roff, sizeof(double) * buf.size(),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (long long r = 0; r < n; r++) {
            if (t) t[r] = buf[r * (1 + sh.ng)];
            if (eta)
                for (int k = 0; k < sh.ng; k++) eta[r * sh.ng + k] = buf[r * (1 + sh.ng) + 1 + k];
        }
    }
    st[scenario].records = 0;
    return push_scen(c, st);
}

static int collect_timing(hsgn_ctx *c);

static int timed_begin(hsgn_ctx *c, hipStream_t s)
{
    if (!c->timing) return HSGN_OK;
    if (c->ev_used + 2 > c->ev.size()) {
        for (int k = 0; k < 256; k++) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    HIPCHK(c, hipEventRecord(c->ev[c->ev_used], s));
    return HSGN_OK;
}

static int timed_end(hsgn_ctx *c, hipStream_t s)
{
    if (!c->timing) return HSGN_OK;
    HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], s));
    c->ev_used += 2;
    return HSGN_OK;
}

static void launch_gauges(hsgn_ctx *c, hipStream_t s)
{
    if (c->ngauge_total <= 0) return;
    unsigned gb = (unsigned)((c->ngauge_total + 63) / 64);
    if (c->mixed)
        gauge_kernel<float, true><<<gb, 64, 0, s>>>(c->d_gauges, c->ngauge_total, c->d_scen, c->f0,
                                                    c->f1, c->fbath, c->prm.eta0, c->prm.dry_tol,
                                                    c->rec);
    else
        gauge_kernel<double, false><<<gb, 64, 0, s>>>(c->d_gauges, c->ngauge_total, c->d_scen, c->q0,
                                                      c->q1, c->bath, c->prm.eta0, c->prm.dry_tol,
                                                      c->rec);
}

// mixed-precision items of one kind (single grids, or patches of patch sets
// with amr) with the class split (A.list set): classified, then the kernel
// without the FP64 edge solve over the items that do not need it and the
// full kernel over the rest.  With fork the few items that need it (each
// runs long, in one round of waves) run on a second stream beside the other
// kernel, joined back into s (also while s is captured into a graph: the
// second stream joins the capture through the fork event); otherwise one
// after the other on s.
static void launch_mixed_split(hsgn_ctx *c, const MarchArgs<float> &A, unsigned n, int *cls,
                               bool amr, hipStream_t s, bool fork)
{
    auto full = [&](hipStream_t st, bool beside) {
        if (amr) launch_march32_amr(A, n, st, beside);
        else launch_march32(A, n, st, beside);
    };
    auto deep = [&](hipStream_t st) {
        if (amr) launch_march32_amr_deep(A, n, st);
        else launch_march32_deep(A, n, st);
    };
    if (!A.list) {
        full(s, false);
        return;
    }
    if (amr) launch_classify32_amr(A, n, cls, s);
    else launch_classify32(A, n, cls, s);
    if (fork) {
        (void)hipEventRecord(c->ev_fork, s);
        (void)hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0);
        full(c->aux_stream, true);
        deep(s);
        (void)hipEventRecord(c->ev_join, c->aux_stream);
        (void)hipStreamWaitEvent(s, c->ev_join, 0);
    } else {
        full(s, false);
        deep(s);
    }
}

// the split's buffers for items [w0, w1) of the context's work table
static void split_args(hsgn_ctx *c, MarchArgs<float> &A, int w0)
{
    if (!c->split) return;
    A.list = c->d_list + 2 * w0;
    A.lcnt = c->d_lcnt;
    A.clsb = c->d_clsb + w0;
}

// step kernels over work items [w0, w1): single grids with the plain
// kernel, patch-set patches [wa, w1) with the patch-set kernel
static void launch_march_range(hsgn_ctx *c, int w0, int wa, int w1, hipStream_t s, bool fork)
{
    if (wa > w0) {
        if (c->mixed) {
            MarchArgs<float> A = march_args<float>(c, c->f0, c->f1, c->fbath, w0, wa);
            split_args(c, A, w0);
            A.latch = c->d_latch;               // single-grid contexts only
            launch_mixed_split(c, A, (unsigned)(wa - w0), c->d_cls + w0, false, s, fork);
        } else
            launch_march64(march_args<double>(c, c->q0, c->q1, c->bath, w0, wa), (unsigned)(wa - w0), s);
    }
    if (w1 > wa) {
        if (c->mixed) {
            MarchArgs<float> A = march_args<float>(c, c->f0, c->f1, c->fbath, wa, w1);
            A.mapped = c->mapped_amr ? 1 : 0;
            split_args(c, A, wa);
            launch_mixed_split(c, A, (unsigned)(w1 - wa), c->d_cls + wa, true, s, fork);
        } else {
            MarchArgs<double> A = march_args<double>(c, c->q0, c->q1, c->bath, wa, w1);
            A.mapped = c->mapped_amr ? 1 : 0;
            launch_march64_amr(A, (unsigned)(w1 - wa), s);
        }
    }
}

static void launch_control(hsgn_ctx *c, int s0, int s1, hipStream_t s)
{
    if (s1 > s0)
        control_kernel<<<(unsigned)(s1 - s0), 256, 0, s>>>(c->d_scen + s0, c->d_sstat + s0, c->clip,
                                                            s1 - s0);
}

// one step of level l (and, recursively, the 4 substeps of every finer
// level) of all patch sets and single grids
static void launch_level(hsgn_ctx *c, int l, double theta, hipStream_t s, bool timed)
{
    const LevelRange &R = c->L[l];
    const double eta0 = c->prm.eta0, dtol = c->prm.dry_tol;
    if (c->mixed) {
        AmrBuffers<float> B = amr_buffers<float>(c, c->f0, c->f1, c->fbath);
        launch_halo_copy32(B, c->d_gc + R.gc0, R.gc1 - R.gc0, s);
        launch_halo_interp32(B, c->d_gi + R.gi0, R.gi1 - R.gi0, theta, eta0, dtol, s);
    } else {
        AmrBuffers<double> B = amr_buffers<double>(c, c->q0, c->q1, c->bath);
        launch_halo_copy64(B, c->d_gc + R.gc0, R.gc1 - R.gc0, s);
        launch_halo_interp64(B, c->d_gi + R.gi0, R.gi1 - R.gi0, theta, eta0, dtol, s);
    }
    if (timed) (void)timed_begin(c, s);
    launch_march_range(c, R.w0, R.wa, R.w1, s, true);
    if (timed) (void)timed_end(c, s);
    launch_control(c, R.s0, R.s1, s);
    if (l + 1 >= c->nlev) return;
    const LevelRange &F = c->L[l + 1];
    launch_fill_zero(c->d_R + 7 * F.e0, 7 * (F.e1 - F.e0), s);
    for (int sub = 0; sub < AMR_RATIO; sub++) {
        launch_level(c, l + 1, (double)sub / AMR_RATIO, s, timed);
        if (c->mixed)
            launch_bflux32(amr_buffers<float>(c, c->f0, c->f1, c->fbath), c->P, c->d_fr + F.fr0,
                           F.fr1 - F.fr0, c->d_E, c->d_R, s);
        else
            launch_bflux64(amr_buffers<double>(c, c->q0, c->q1, c->bath), c->P, c->d_fr + F.fr0,
                           F.fr1 - F.fr0, c->d_E, c->d_R, s);
    }
    if (c->mixed) {
        AmrBuffers<float> B = amr_buffers<float>(c, c->f0, c->f1, c->fbath);
        launch_reflux32(B, c->P, c->d_rf + R.rf0, R.rf1 - R.rf0, c->d_R, c->d_rclip + R.rf0, s);
        launch_avgdown32(B, c->d_av + F.av0, F.av1 - F.av0, false, s);
    } else {
        AmrBuffers<double> B = amr_buffers<double>(c, c->q0, c->q1, c->bath);
        launch_reflux64(B, c->P, c->d_rf + R.rf0, R.rf1 - R.rf0, c->d_R, c->d_rclip + R.rf0, s);
        launch_avgdown64(B, c->d_av + F.av0, F.av1 - F.av0, false, s);
    }
}

// the bottom part of the split step's classes for the single-grid items of
// every level, after a bathymetry or work-table change
static void refresh_static_classes(hsgn_ctx *c)
{
    if (!c->split || !c->clsb_dirty) return;
    for (int l = 0; l < c->nlev; l++) {
        const LevelRange &R = c->L[l];
        if (R.wa > R.w0)
            launch_static_class32(march_args<float>(c, c->f0, c->f1, c->fbath, R.w0, R.wa),
                                  (unsigned)(R.wa - R.w0), c->d_clsb + R.w0, c->stream);
        if (R.w1 > R.wa)
            launch_static_class32_amr(march_args<float>(c, c->f0, c->f1, c->fbath, R.wa, R.w1),
                                      (unsigned)(R.w1 - R.wa), c->d_clsb + R.wa, c->stream);
    }
    c->clsb_dirty = false;
}

// one step attempt of every scenario
static int launch_attempt(hsgn_ctx *c)
{
    refresh_static_classes(c);
    if (!c->any_amr) {
        if ((c->timing && timed_begin(c, c->stream))) return HSGN_EDEVICE;
        launch_march_range(c, 0, (int)c->work.size(), (int)c->work.size(), c->stream, true);
        if ((c->timing && timed_end(c, c->stream))) return HSGN_EDEVICE;
        launch_control(c, 0, c->nslot, c->stream);
        launch_gauges(c, c->stream);
        HIPCHK(c, hipGetLastError());
        return HSGN_OK;
    }
    // patch sets: the whole level-0 step with its substeps, replayed from a
    // captured graph (captured on a private stream, launched on the
    // context's); with timing on, direct launches with the step kernels timed
    if (!c->timing && !c->graph_failed && !c->graph_valid) {
        if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (ok) {
            launch_level(c, 0, 0.0, c->cap_stream, false);
            launch_gauges(c, c->cap_stream);
            ok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && g;
        }
        if (ok) ok = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->graph_valid = ok;
        c->graph_failed = !ok;
    }
    if (!c->timing && c->graph_valid) {
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
        return HSGN_OK;
    }
    launch_level(c, 0, 0.0, c->stream, c->timing);
    launch_gauges(c, c->stream);
    HIPCHK(c, hipGetLastError());
    return HSGN_OK;
}

int hsgn_advance(hsgn_ctx *c, double dt, int n_steps)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (n_steps < 0) return fail(c, HSGN_EINVAL, "negative step count");
    if (n_steps == 0) return HSGN_OK;
    int rc = ensure_prepared(c);
    if (rc) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    // dt > 0: one fixed step for all scenarios; dt == 0: adaptive steps;
    // dt < 0: each scenario keeps the fixed step stored in its clock
    bool adaptive = dt == 0.0;
    bool per_scen = dt < 0.0;
    if (adaptive && c->any_amr)
        return fail(c, HSGN_ENOTSUP, "patch sets advance with fixed steps (dt != 0)");
    bool need_dt0 = false;
    const int nscen = (int)c->scen.size();
    for (int s = 0; s < nscen; s++) {
        if (st[s].err) return fail(c, st[s].err, "scenario in error state");
        if (per_scen && !(st[s].dt > 0.0))
            return fail(c, HSGN_EINVAL, "per-scenario fixed step not set (hsgn_set_clock)");
        st[s].adaptive = adaptive ? 1 : 0;
        st[s].dt_fixed = adaptive ? 0.0 : (per_scen ? st[s].dt : dt);
        if (!adaptive && !per_scen) st[s].dt = dt;
        else if (adaptive && !(st[s].dt > 0.0)) need_dt0 = true;
        st[s].target = st[s].steps + n_steps;
        st[s].active = 1;
        st[s].streak = 0;
        st[s].rx_bits = 0; st[s].ry_bits = 0;
        // finer levels of a patch set: 4^l substeps of dt / 4^l
        const ScenHost &sh = c->scen[s];
        long long k = 1;
        for (size_t l = 1; l < sh.slot.size(); l++) {
            k *= AMR_RATIO;
            ScenState &f = st[sh.slot[l]];
            if (f.err) return fail(c, f.err, "scenario in error state");
            f.adaptive = 0;
            f.dt = st[s].dt_fixed / (double)k;
            f.dt_fixed = f.dt;
            f.target = f.steps + (long long)n_steps * k;
            f.active = 1;
            f.streak = 0;
            f.rx_bits = 0; f.ry_bits = 0;
        }
    }
    if ((rc = push_scen(c, st))) return rc;
    if (need_dt0) {
        HIPCHK(c, hipMemsetAsync(c->d_slots, 0, sizeof(unsigned long long) * nscen, c->stream));
        HIPCHK(c, hipMemsetAsync(c->d_err, 0, sizeof(int), c->stream));
        for (size_t pid = 0; pid < c->patches.size(); pid++) {
            const PatchInfo &p = c->patches[pid];
            if (st[p.scen].dt > 0.0) continue;
            long long n = (long long)p.nx * p.ny;
            const uint8_t *m = st[p.scen].cur ? c->m1 : c->m0;
            if (c->mixed)
                initdt_kernel<float, true><<<nblk(n), 256, 0, c->stream>>>(
                    p, c->P, st[p.scen].cur ? c->f1 : c->f0, c->fbath, m, c->d_slots + p.scen,
                    c->d_err);
            else
                initdt_kernel<double, false><<<nblk(n), 256, 0, c->stream>>>(
                    p, c->P, st[p.scen].cur ? c->q1 : c->q0, c->bath, m, c->d_slots + p.scen,
                    c->d_err);
        }
        initdt_finish<<<(unsigned)((nscen + 63) / 64), 64, 0, c->stream>>>(c->d_scen, c->d_sstat,
                                                                           c->d_slots, nscen);
        HIPCHK(c, hipGetLastError());
        int err = 0;
        HIPCHK(c, hipMemcpyAsync(&err, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (err) return fail(c, err, "initial step: state not hyperbolic");
    }
    if ((rc = ensure_gauges(c, st, (long long)n_steps + 256))) return rc;
    // the first attempt classifies (masks or bathymetry may have changed
    // since the last advance); later ones only after a latch
    if (c->d_latch) {
        set_flag_kernel<<<1, 64, 0, c->stream>>>(c->d_latch, 1);
        HIPCHK(c, hipGetLastError());
    }
    long long attempts = n_steps, budget = (long long)n_steps + 4096;
    while (attempts > 0) {
        for (long long a = 0; a < attempts; a++) {
            if ((rc = launch_attempt(c))) return rc;
            if (c->timing && c->ev_used >= 8192 && (rc = collect_timing(c))) return rc;
        }
        budget -= attempts;
        if ((rc = pull_scen(c, st))) return rc;
        long long left = 0;
        for (int s = 0; s < nscen; s++)
            if (st[s].active && !st[s].err) left = std::max(left, st[s].target - st[s].steps);
        if (left > 0 && budget > 0 && !c->any_amr) {
            if ((rc = ensure_gauges(c, st, left + 256))) return rc;
            attempts = std::min(left, budget);
        } else {
            attempts = 0;
        }
    }
    for (int s = 0; s < nscen; s++) {
        int err = st[s].err;
        for (size_t l = 1; l < c->scen[s].slot.size() && !err; l++) err = st[c->scen[s].slot[l]].err;
        if (err) return fail(c, err, std::string("scenario ") + std::to_string(s) + ": " + hsgn_strerror(err));
        if (st[s].steps < st[s].target) return fail(c, HSGN_ECFL, "too many rejected steps");
    }
    return HSGN_OK;
}

// Autotuning of the tile height, per refinement level: every candidate is
// timed with step-kernel launches over that level's patches on the current
// state.  The launches write only the spare state buffer (no clock slot is
// swapped), and the clock slots are restored afterwards, so the state does
// not advance.
int hsgn_autotune(hsgn_ctx *c, int trials, int *rows)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (trials < 1 || trials > 100) return fail(c, HSGN_EINVAL, "trials must be 1..100");
    int rc = ensure_prepared(c);
    if (rc) return rc;
    std::vector<ScenState> saved, st;
    if ((rc = pull_scen(c, saved))) return rc;
    st = saved;
    for (ScenState &x : st) {
        x.active = 1;
        x.err = 0;
    }
    if ((rc = push_scen(c, st))) return rc;
    static const int cand[] = {2, 4, 6, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64};
    // per level: these heights and the cost model's own choice, ascending
    // (the model lands between them for grids that fill the chip in one round)
    std::vector<std::vector<int>> cands(c->nlev);
    for (int l = 0; l < c->nlev; l++) {
        cands[l].assign(std::begin(cand), std::end(cand));
        const int m = model_rows(c, l);
        if (std::find(cands[l].begin(), cands[l].end(), m) == cands[l].end()) {
            cands[l].push_back(m);
            std::sort(cands[l].begin(), cands[l].end());
        }
    }
    // scratch work table, packed items and clip slots for the largest
    // candidate table
    std::vector<WorkItem> wk;
    std::vector<PackedItem> pk;
    std::vector<ScenStatic> ss;
    std::vector<LevelRange> L = c->L;
    size_t wmax = 1, pmax = 1;
    for (int l = 0; l < c->nlev; l++)
        for (int th : cands[l]) {
            std::vector<int> thl = c->th_level;
            thl[l] = th;
            build_work(c, thl, wk, pk, ss, L);
            wmax = std::max(wmax, wk.size());
            pmax = std::max(pmax, pk.size());
        }
    WorkItem *dwork = nullptr;
    PackedItem *dpacks = nullptr;
    double *dclip = nullptr;
    int *dlist = nullptr, *dclsb = nullptr, *dcls = nullptr;
    unsigned *dlcnt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (dwork) (void)hipFree(dwork);
        if (dpacks) (void)hipFree(dpacks);
        if (dclip) (void)hipFree(dclip);
        if (dlist) (void)hipFree(dlist);
        if (dlcnt) (void)hipFree(dlcnt);
        if (dcls) (void)hipFree(dcls);
        if (dclsb) (void)hipFree(dclsb);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&dwork, sizeof(WorkItem) * wmax) != hipSuccess ||
        hipMalloc(&dpacks, sizeof(PackedItem) * pmax) != hipSuccess ||
        hipMalloc(&dclip, sizeof(double) * wmax) != hipSuccess ||
        hipMalloc(&dlist, sizeof(int) * 2 * wmax) != hipSuccess ||
        hipMalloc(&dlcnt, sizeof(unsigned) * 2) != hipSuccess ||
        hipMalloc(&dcls, sizeof(int) * wmax) != hipSuccess ||
        hipMalloc(&dclsb, sizeof(int) * wmax) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(c, HSGN_ENOMEM, "autotune scratch");
    }
    std::vector<int> best = c->th_level;
    for (int l = 0; l < c->nlev; l++) {
        int maxny = 0;
        for (const PatchInfo &p : c->patches)
            if (p.level == l) maxny = std::max(maxny, p.ny);
        // ghost frames of patch sets from the current states
        const LevelRange &R = c->L[l];
        if (c->mixed) {
            AmrBuffers<float> B = amr_buffers<float>(c, c->f0, c->f1, c->fbath);
            launch_halo_copy32(B, c->d_gc + R.gc0, R.gc1 - R.gc0, c->stream);
            launch_halo_interp32(B, c->d_gi + R.gi0, R.gi1 - R.gi0, 1.0, c->prm.eta0,
                                 c->prm.dry_tol, c->stream);
        } else {
            AmrBuffers<double> B = amr_buffers<double>(c, c->q0, c->q1, c->bath);
            launch_halo_copy64(B, c->d_gc + R.gc0, R.gc1 - R.gc0, c->stream);
            launch_halo_interp64(B, c->d_gi + R.gi0, R.gi1 - R.gi0, 1.0, c->prm.eta0,
                                 c->prm.dry_tol, c->stream);
        }
        double best_ms = -1.0;
        int prev = 0;
        for (int th : cands[l]) {
            if (prev >= maxny) break;           // taller tiles give the same work table
            prev = th;
            std::vector<int> thl = c->th_level;
            thl[l] = th;
            build_work(c, thl, wk, pk, ss, L);
            const LevelRange &Q = L[l];
            int n = Q.w1 - Q.w0;
            if (n <= 0) continue;
            if (!packs_ok(c, wk, pk)) {
                cleanup();
                return fail(c, HSGN_EINVAL, "internal table check: packed items");
            }
            if (hipMemcpyAsync(dwork, wk.data() + Q.w0, sizeof(WorkItem) * n, hipMemcpyHostToDevice,
                               c->stream) != hipSuccess ||
                (!pk.empty() && hipMemcpyAsync(dpacks, pk.data(), sizeof(PackedItem) * pk.size(),
                                               hipMemcpyHostToDevice, c->stream) != hipSuccess)) {
                cleanup();
                return fail(c, HSGN_EDEVICE, "autotune upload");
            }
            int na = Q.wa - Q.w0;    // single-grid items first, then patch-set items
            auto launch = [&]() {
                if (na > 0) {
                    if (c->mixed) {
                        MarchArgs<float> A = march_args<float>(c, c->f0, c->f1, c->fbath, 0, na);
                        A.work = dwork; A.packs = dpacks; A.clip_slots = dclip;
                        if (c->split) {
                            A.list = dlist;
                            A.lcnt = dlcnt;
                            A.clsb = dclsb;
                        }
                        launch_mixed_split(c, A, (unsigned)na, dcls, false, c->stream, true);
                    } else {
                        MarchArgs<double> A = march_args<double>(c, c->q0, c->q1, c->bath, 0, na);
                        A.work = dwork; A.packs = dpacks; A.clip_slots = dclip;
                        launch_march64(A, (unsigned)na, c->stream);
                    }
                }
                if (n > na) {
                    if (c->mixed) {
                        MarchArgs<float> A = march_args<float>(c, c->f0, c->f1, c->fbath, 0, n - na);
                        A.work = dwork + na; A.packs = dpacks; A.clip_slots = dclip + na;
                        A.mapped = c->mapped_amr ? 1 : 0;
                        if (c->split) {
                            A.list = dlist + 2 * na;
                            A.lcnt = dlcnt;
                            A.clsb = dclsb + na;
                        }
                        launch_mixed_split(c, A, (unsigned)(n - na), dcls + na, true, c->stream, true);
                    } else {
                        MarchArgs<double> A = march_args<double>(c, c->q0, c->q1, c->bath, 0, n - na);
                        A.work = dwork + na; A.packs = dpacks; A.clip_slots = dclip + na;
                        A.mapped = c->mapped_amr ? 1 : 0;
                        launch_march64_amr(A, (unsigned)(n - na), c->stream);
                    }
                }
            };
            if (na > 0 && c->split) {
                MarchArgs<float> A = march_args<float>(c, c->f0, c->f1, c->fbath, 0, na);
                A.work = dwork;
                launch_static_class32(A, (unsigned)na, dclsb, c->stream);
            }
            if (n > na && c->split) {
                MarchArgs<float> A = march_args<float>(c, c->f0, c->f1, c->fbath, 0, n - na);
                A.work = dwork + na;
                A.packs = dpacks;
                launch_static_class32_amr(A, (unsigned)(n - na), dclsb + na, c->stream);
            }
            launch();                                   // warm-up
            (void)hipEventRecord(e0, c->stream);
            for (int t = 0; t < trials; t++) launch();
            (void)hipEventRecord(e1, c->stream);
            if (hipEventSynchronize(e1) != hipSuccess) {
                cleanup();
                return fail(c, HSGN_EDEVICE, "autotune timing");
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (best_ms < 0.0 || ms < best_ms) { best_ms = ms; best[l] = th; }
        }
    }
    cleanup();
    HIPCHK(c, hipGetLastError());
    if ((rc = push_scen(c, saved))) return rc;
    // the chosen tile heights
    if ((rc = install_work(c, best))) return rc;
    if (rows)
        for (int l = 0; l < c->nlev; l++) rows[l] = best[l];
    return HSGN_OK;
}

int hsgn_diagnostics(hsgn_ctx *c, int scenario, hsgn_diag *d)
{
    if (!c || !c->finalized || !d) return fail(c, HSGN_EINVAL, "bad arguments");
    if (scenario < 0 || scenario >= (int)c->scen.size()) return fail(c, HSGN_EINVAL, "bad scenario");
    int rc = ensure_prepared(c);
    if (rc) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    memset(d, 0, sizeof(*d));
    const ScenHost &sh = c->scen[scenario];
    const ScenState &s = st[scenario];
    double mass = 0.0, clip = 0.0, maxc = 0.0;
    unsigned long long cnt_h[2] = {0, 0};
    long long updates = 0;
    for (size_t l = 0; l < sh.lev.size(); l++) {
        const ScenState &sl = st[sh.slot[l]];
        clip += sl.clip_total;
        maxc = std::max(maxc, sl.max_courant);
        for (int pid : sh.lev[l]) {
            const PatchInfo &p = c->patches[pid];
            long long n = (long long)p.nx * p.ny;
            updates += sl.steps * n;
            const uint8_t *m = sl.cur ? c->m1 : c->m0;
            HIPCHK(c, hipMemsetAsync(c->d_cnt, 0, sizeof(unsigned long long) * 2, c->stream));
            count_kernel<<<nblk(n), 256, 0, c->stream>>>(p, m, c->d_cnt);
            unsigned long long ch[2];
            HIPCHK(c, hipMemcpyAsync(ch, c->d_cnt, sizeof(ch), hipMemcpyDeviceToHost, c->stream));
            if (l == 0) {
                // the mass of a patch set is that of level 0 (finer levels are
                // averaged onto it after every level-0 step)
                if (c->mixed)
                    mass_kernel<float, true><<<1, 1024, 0, c->stream>>>(p, sl.cur ? c->f1 : c->f0,
                                                                        c->fbath, c->prm.eta0,
                                                                        c->d_mass);
                else
                    mass_kernel<double, false><<<1, 1024, 0, c->stream>>>(p, sl.cur ? c->q1 : c->q0,
                                                                          c->bath, c->prm.eta0,
                                                                          c->d_mass);
                double pm = 0.0;
                HIPCHK(c, hipMemcpyAsync(&pm, c->d_mass, sizeof(double), hipMemcpyDeviceToHost,
                                         c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                mass += pm * p.dx * p.dy;
            }
            HIPCHK(c, hipStreamSynchronize(c->stream));
            cnt_h[0] += ch[0];
            cnt_h[1] += ch[1];
        }
    }
    if (!c->h_rf.empty()) {
        std::vector<double> rcl(c->h_rf.size());
        HIPCHK(c, hipMemcpyAsync(rcl.data(), c->d_rclip, sizeof(double) * rcl.size(),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < rcl.size(); k++) {
            int slot = c->patches[c->h_rf[k].cp].scen;
            for (int sl : sh.slot)
                if (sl == slot) clip += rcl[k];
        }
    }
    d->mass = mass;
    d->clipped_mass = clip;
    d->max_courant = maxc;
    d->last_courant = s.courant;
    d->steps = s.steps;
    d->rejected = s.rejects;
    d->cell_updates = updates;
    d->n_swe_cells = (long long)cnt_h[0];
    d->n_breaking = (long long)cnt_h[1];
    return HSGN_OK;
}

int hsgn_get_clock(hsgn_ctx *c, int scenario, double *t, double *dt_next, long long *steps)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (scenario < 0 || scenario >= (int)c->scen.size()) return fail(c, HSGN_EINVAL, "bad scenario");
    std::vector<ScenState> st;
    int rc = pull_scen(c, st);
    if (rc) return rc;
    if (t) *t = st[scenario].t;
    if (dt_next) *dt_next = st[scenario].dt;
    if (steps) *steps = st[scenario].steps;
    return HSGN_OK;
}

int hsgn_set_clock(hsgn_ctx *c, int scenario, double t, double dt_next, long long steps)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (scenario < 0 || scenario >= (int)c->scen.size()) return fail(c, HSGN_EINVAL, "bad scenario");
    std::vector<ScenState> st;
    int rc = pull_scen(c, st);
    if (rc) return rc;
    const ScenHost &sh = c->scen[scenario];
    long long k = 1;
    for (size_t l = 0; l < sh.slot.size(); l++) {
        ScenState &x = st[sh.slot[l]];
        x.t = t;
        x.dt = dt_next > 0.0 ? dt_next / (double)k : 0.0;
        x.steps = steps * k;
        x.err = 0;
        k *= AMR_RATIO;
    }
    return push_scen(c, st);
}

static int collect_timing(hsgn_ctx *c)
{
    if (c->ev_used == 0) return HSGN_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
        c->timed_ms += ms;
        c->timed_launches += 1;
    }
    c->ev_used = 0;
    return HSGN_OK;
}

int hsgn_set_timing(hsgn_ctx *c, int on)
{
    if (!c) return HSGN_EINVAL;
    int rc = collect_timing(c);
    if (rc) return rc;
    c->timing = on != 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return HSGN_OK;
}

int hsgn_get_timing(hsgn_ctx *c, double *step_kernel_ms, long long *launches)
{
    if (!c) return HSGN_EINVAL;
    int rc = collect_timing(c);
    if (rc) return rc;
    if (step_kernel_ms) *step_kernel_ms = c->timed_ms;
    if (launches) *launches = c->timed_launches;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return HSGN_OK;
}

int hsgn_work_items(hsgn_ctx *c, int *n)
{
    if (!c || !c->finalized || !n) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    *n = (int)c->work.size();
    return HSGN_OK;
}

// ---------------------------------------------------------------------------
// hsgn_advance_static: one FP64 single grid advanced without any allocation.
// Its working memory (the spare state buffer, both mask buffers, the patch,
// clock and work tables, the clipped-mass slots) lives in the file-scope
// array below, one copy per device, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: the device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is used.

constexpr size_t HSGN_STATIC_BYTES = (size_t)HSGN_STATIC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[HSGN_STATIC_BYTES];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
std::once_flag g_scratch_once[STATIC_MAX_DEVICES];
unsigned char *g_scratch_ptr[STATIC_MAX_DEVICES];
hipError_t g_scratch_err[STATIC_MAX_DEVICES];

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// byte offsets of the working memory's parts for ncell cells and nwork items
struct StaticLayout {
    size_t q1, m0, m1, patch, sstat, scen, work, clip, total;
};

StaticLayout static_layout(long long ncell, long long nwork)
{
    StaticLayout L;
    size_t o = 0;
    L.q1 = o;    o = align256(o + sizeof(double) * 7 * (size_t)ncell);
    L.m0 = o;    o = align256(o + (size_t)ncell);
    L.m1 = o;    o = align256(o + (size_t)ncell);
    L.patch = o; o = align256(o + sizeof(PatchInfo));
    L.sstat = o; o = align256(o + sizeof(ScenStatic));
    L.scen = o;  o = align256(o + sizeof(ScenState));
    L.work = o;  o = align256(o + sizeof(WorkItem) * (size_t)nwork);
    L.clip = o;  o = align256(o + sizeof(double) * (size_t)nwork);
    L.total = o;
    return L;
}
}  // namespace

// the patch, clock and work tables of the grid, written from kernel
// arguments (no host buffer, no memset: safe under graph capture)
__global__ void static_setup_kernel(PatchInfo pi, ScenStatic ss, ScenState st, PatchInfo *dp,
                                    ScenStatic *dss, ScenState *dst, WorkItem *work, double *clip,
                                    int nwork, int nstrips, int th)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k == 0) { *dp = pi; *dss = ss; *dst = st; }
    if (k < nwork) {
        const int r0 = (k / nstrips) * th;
        work[k] = WorkItem{0, (k % nstrips) * 60, r0, min(th, pi.ny - r0)};
        clip[k] = 0.0;
    }
}

// Q^n back into the caller's buffer when the last accepted step left it in
// the spare one
__global__ void static_copyback_kernel(const ScenState *st, const double *q1, double *q,
                                       long long n)
{
    if (!st->cur) return;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        q[i] = q1[i];
}

int hsgn_advance_static(const hsgn_params *p, void *hip_stream, int nx, int ny, double dx,
                        double dy, const int bc[4], const double *b, double *q, double dt,
                        int n_steps, long long *steps_done)
{
    if (steps_done) *steps_done = 0;
    if (!p || !bc || !b || !q) return HSGN_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    if (p->precision != 0) return HSGN_ENOTSUP;
    if (nx < 4 || ny < 4 || !(dx > 0) || !(dy > 0) || !(dt > 0) || n_steps < 0)
        return HSGN_EINVAL;
    for (int k = 0; k < 4; k++)
        if (bc[k] < 0 || bc[k] > 2) return HSGN_EINVAL;
    if ((bc[0] == HSGN_BC_PERIODIC) != (bc[1] == HSGN_BC_PERIODIC) ||
        (bc[2] == HSGN_BC_PERIODIC) != (bc[3] == HSGN_BC_PERIODIC))
        return HSGN_EINVAL;
    const long long ncell = (long long)nx * ny;
    if (ncell > (long long)(HSGN_STATIC_BYTES / 58)) return HSGN_ESCRATCH;
    // tile height: the library's cost model for one FP64 grid (1024
    // resident wavefronts), unless the caller fixes it
    const long long nstrips = (nx + 59) / 60, slots = 1024;
    int th = p->tile_rows > 0 ? p->tile_rows : 64;
    if (p->tile_rows <= 0) {
        long long best = -1;
        for (int t = 64; t >= 8; t--) {
            const long long cost = ((nstrips * ((ny + t - 1) / t) + slots - 1) / slots) * (t + 4);
            if (best < 0 || cost < best) { best = cost; th = t; }
        }
    }
    const long long nwork = nstrips * ((ny + th - 1) / th);
    const StaticLayout L = static_layout(ncell, nwork);
    if (L.total > HSGN_STATIC_BYTES) return HSGN_ESCRATCH;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES)
        return HSGN_EDEVICE;
    std::call_once(g_scratch_once[dev], [dev]() {
        void *ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = (unsigned char *)ptr;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev]) return HSGN_EDEVICE;
    unsigned char *base = g_scratch_ptr[dev];
    hipStream_t s = (hipStream_t)hip_stream;

    PatchInfo pi;
    memset(&pi, 0, sizeof(pi));
    pi.nx = nx; pi.ny = ny; pi.pitch = nx; pi.scen = 0;
    for (int k = 0; k < 4; k++) pi.bc[k] = bc[k];
    pi.dx = dx; pi.dy = dy;
    pi.qoff = 0; pi.coff = 0; pi.plane = ncell; pi.eoff = -1;
    pi.level = 0; pi.frame = 0; pi.metric = nullptr;
    ScenStatic ss;
    ss.dx = dx; ss.dy = dy; ss.cfl = p->cfl; ss.cfl_max = p->cfl_max;
    ss.w0 = 0; ss.w1 = (int)nwork;
    ScenState st;
    memset(&st, 0, sizeof(st));
    st.dt = dt; st.dt_fixed = dt;
    st.target = n_steps;
    st.active = n_steps > 0 ? 1 : 0;

    double *q1 = (double *)(base + L.q1);
    uint8_t *m0 = base + L.m0, *m1 = base + L.m1;
    PatchInfo *dp = (PatchInfo *)(base + L.patch);
    ScenStatic *dss = (ScenStatic *)(base + L.sstat);
    ScenState *dst = (ScenState *)(base + L.scen);
    WorkItem *work = (WorkItem *)(base + L.work);
    double *clip = (double *)(base + L.clip);

    static_setup_kernel<<<nblk(nwork), 256, 0, s>>>(pi, ss, st, dp, dss, dst, work, clip,
                                                    (int)nwork, (int)nstrips, th);
    mask_kernel<double><<<nblk(ncell), 256, 0, s>>>(pi, b, m0, m1, p->eta0, p->h_star, p->nbr_n);
    MarchArgs<double> A;
    A.P = step_params(p);
    A.patches = dp;
    A.work = work;
    A.packs = nullptr;
    A.q0 = q; A.q1 = q1;
    A.bath = b;
    A.m0 = m0; A.m1 = m1;
    A.scen = dst;
    A.clip_slots = clip;
    A.eflux = nullptr;
    A.list = nullptr; A.lcnt = nullptr; A.clsb = nullptr; A.latch = nullptr;
    A.sponge = 0; A.mapped = 0;
    A.nwork = (int)nwork;
    for (int a = 0; a < n_steps; a++) {
        launch_march64(A, (unsigned)nwork, s);
        control_kernel<<<1, 256, 0, s>>>(dst, dss, clip, 1);
    }
    static_copyback_kernel<<<nblk(std::min<long long>(7 * ncell, 1 << 22)), 256, 0, s>>>(
        dst, q1, q, 7 * ncell);
    if (hipGetLastError() != hipSuccess) return HSGN_EDEVICE;
    ScenState out;
    if (hipMemcpyAsync(&out, dst, sizeof(out), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return HSGN_EDEVICE;
    if (steps_done) *steps_done = out.steps;
    return out.err;
}

int hsgn_destroy(hsgn_ctx *c)
{
    if (!c) return HSGN_EINVAL;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_device(c);
    delete c;
    return HSGN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// regridding: flags on level l, clusters, a new context with the rebuilt
// level l+1, the state moved across on the device, then the new context takes
// the place of the old one behind the caller's handle.

namespace {

struct RgBox {
    int i0, i1, j0, j1;     // half-open, in cells of the flagged patch
};

// clusters of the flags F[ny][nx] (Berger-Rigoutsos, rules in hsgn.h)
void rg_cluster(const std::vector<uint8_t> &F, int NX, int i0, int i1, int j0, int j1,
                double cutoff, int max_side, std::vector<RgBox> &out)
{
    int a0 = i1, a1 = i0 - 1, b0 = j1, b1 = j0 - 1;
    long long n = 0;
    for (int j = j0; j < j1; j++)
        for (int i = i0; i < i1; i++)
            if (F[(size_t)j * NX + i]) {
                n++;
                a0 = std::min(a0, i); a1 = std::max(a1, i);
                b0 = std::min(b0, j); b1 = std::max(b1, j);
            }
    if (n == 0) return;
    i0 = a0; i1 = a1 + 1; j0 = b0; j1 = b1 + 1;
    const int nx = i1 - i0, ny = j1 - j0;
    int dim = -1, cut = 0;
    if ((double)n >= cutoff * (double)((long long)nx * ny)) {
        if (nx <= max_side && ny <= max_side) {
            out.push_back({i0, i1, j0, j1});
            return;
        }
        if (nx >= ny) { dim = 0; cut = nx / 2; } else { dim = 1; cut = ny / 2; }
    } else {
        std::vector<long long> S[2];
        S[0].assign(nx, 0);
        S[1].assign(ny, 0);
        for (int j = j0; j < j1; j++)
            for (int i = i0; i < i1; i++)
                if (F[(size_t)j * NX + i]) { S[0][i - i0]++; S[1][j - j0]++; }
        const int Ls[2] = {nx, ny};
        // (a) an empty column or row, nearest the middle
        long long bk0 = 0;
        int bd = 0, bk = 0;
        bool found = false;
        for (int d = 0; d < 2; d++)
            for (int k = 1; k < Ls[d] - 1; k++)
                if (S[d][k] == 0) {
                    long long k0 = std::llabs(2LL * k - (Ls[d] - 1));
                    if (!found || k0 < bk0 || (k0 == bk0 && (d < bd || (d == bd && k < bk)))) {
                        found = true; bk0 = k0; bd = d; bk = k;
                    }
                }
        if (found) {
            dim = bd; cut = bk;
        } else {
            // (b) the strongest sign change of the second difference
            long long bs = 0, bm = 0;
            for (int d = 0; d < 2; d++) {
                const int L = Ls[d];
                if (L < 4) continue;
                auto lap = [&](int k) { return S[d][k - 1] - 2 * S[d][k] + S[d][k + 1]; };
                for (int k = 1; k < L - 2; k++) {
                    const long long a = lap(k), b = lap(k + 1);
                    if (a * b < 0) {
                        const long long st = std::llabs(b - a);
                        const long long mid = std::llabs(2LL * (k + 1) - L);
                        if (!found || st > bs || (st == bs && (mid < bm || (mid == bm &&
                            (d < bd || (d == bd && k < bk)))))) {
                            found = true; bs = st; bm = mid; bd = d; bk = k;
                        }
                    }
                }
            }
            if (found) {
                dim = bd; cut = bk + 1;
            } else if (nx >= ny) {
                dim = 0; cut = nx / 2;
            } else {
                dim = 1; cut = ny / 2;
            }
        }
    }
    if (dim == 0) {
        rg_cluster(F, NX, i0, i0 + cut, j0, j1, cutoff, max_side, out);
        rg_cluster(F, NX, i0 + cut, i1, j0, j1, cutoff, max_side, out);
    } else {
        rg_cluster(F, NX, i0, i1, j0, j0 + cut, cutoff, max_side, out);
        rg_cluster(F, NX, i0, i1, j0 + cut, j1, cutoff, max_side, out);
    }
}

// bilinear interpolant of the level-0 bathymetry B[NY][NX] at the centres of
// a level-`level` box (level-`level` cells I0.., J0..)
void rg_topo(const std::vector<double> &B, int NX, int NY, int level, int nx, int ny, int I0,
             int J0, std::vector<double> &out)
{
    out.resize((size_t)nx * ny);
    const double sc = (double)(1LL << (2 * level));
    for (int j = 0; j < ny; j++) {
        const double fy = ((double)(J0 + j) + 0.5) / sc - 0.5;
        const int jj = std::min(std::max((int)std::floor(fy), 0), NY - 2);
        const double s = std::min(std::max(fy - jj, 0.0), 1.0);
        for (int i = 0; i < nx; i++) {
            const double fx = ((double)(I0 + i) + 0.5) / sc - 0.5;
            const int ii = std::min(std::max((int)std::floor(fx), 0), NX - 2);
            const double t = std::min(std::max(fx - ii, 0.0), 1.0);
            const double *r0 = &B[(size_t)jj * NX], *r1 = &B[(size_t)(jj + 1) * NX];
            out[(size_t)j * nx + i] = (r0[ii] * (1.0 - t) + r0[ii + 1] * t) * (1.0 - s) +
                                      (r1[ii] * (1.0 - t) + r1[ii + 1] * t) * s;
        }
    }
}

template <class T>
int rg_upload(hsgn_ctx *c, T **d, const std::vector<T> &h)
{
    *d = nullptr;
    if (h.empty()) return HSGN_OK;
    HIPCHK(c, hipMalloc(d, sizeof(T) * h.size()));
    HIPCHK(c, hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return HSGN_OK;
}

// the state of the new context n from the old one c (buffers of the current
// step of every old patch, buffer 0 of the new context)
template <class S, bool MIXED>
int rg_transfer(hsgn_ctx *c, hsgn_ctx *n, const std::vector<ScenState> &st_old,
                const std::vector<std::pair<int, int>> &kept,
                const std::vector<std::pair<int, int>> &fresh_parent,
                const std::vector<int> &old_fine, int level)
{
    S *oq0 = MIXED ? (S *)c->f0 : (S *)c->q0, *oq1 = MIXED ? (S *)c->f1 : (S *)c->q1;
    const S *ob = MIXED ? (const S *)c->fbath : (const S *)c->bath;
    S *nq = MIXED ? (S *)n->f0 : (S *)n->q0;
    const S *nb = MIXED ? (const S *)n->fbath : (const S *)n->bath;
    auto old_rec = [&](int op, const PatchInfo &dst, int si0, int sj0, int di0, int dj0, int w,
                       int h, long long c0) {
        const PatchInfo &src = c->patches[op];
        const int cur = st_old[src.scen].cur;
        RegridCopy<S> r;
        memset(&r, 0, sizeof(r));
        r.src = src; r.dst = dst;
        r.sq = cur ? oq1 : oq0;
        r.sb = ob;
        r.sm = cur ? c->m1 : c->m0;
        r.si0 = si0; r.sj0 = sj0; r.di0 = di0; r.dj0 = dj0;
        r.nx = w; r.ny = h; r.c0 = c0;
        return r;
    };
    // kept patches: whole interiors
    std::vector<RegridCopy<S>> K;
    long long tk = 0;
    for (auto &pr : kept) {
        const PatchInfo &s = c->patches[pr.first];
        K.push_back(old_rec(pr.first, n->patches[pr.second], 0, 0, 0, 0, s.nx, s.ny, tk));
        tk += (long long)s.nx * s.ny;
    }
    // the old level-(l+1) patches by bucket: a new patch meets only those of
    // the buckets it reaches, taken in the order of old_fine
    LevelIndex oidx;
    std::vector<int> opos(c->patches.size(), -1);
    if (!old_fine.empty()) {
        const ScenHost &sh = c->scen[c->slot_scen[c->patches[old_fine[0]].scen]];
        long long fl = 1;
        for (int k = 0; k <= level; k++) fl *= AMR_RATIO;
        oidx.init(c, (long long)sh.NX * fl, (long long)sh.NY * fl);
        for (size_t k = 0; k < old_fine.size(); k++) {
            oidx.add(old_fine[k]);
            opos[old_fine[k]] = (int)k;
        }
    }
    std::vector<int> near;
    // new patches from their parents, then old level-(l+1) overlaps
    std::vector<RegridInterp> I;
    std::vector<RegridCopy<S>> O;
    long long ti = 0, to = 0;
    for (auto &fp : fresh_parent) {
        const int f = fp.first, cp = fp.second;
        RegridInterp r;
        memset(&r, 0, sizeof(r));
        r.fine = n->patches[f];
        r.coarse = n->patches[cp];
        r.ci0 = n->pI0[f] / AMR_RATIO - n->pI0[cp];
        r.cj0 = n->pJ0[f] / AMR_RATIO - n->pJ0[cp];
        if (r.ci0 < 1 || r.cj0 < 1 || r.ci0 + r.fine.nx / AMR_RATIO > r.coarse.nx - 1 ||
            r.cj0 + r.fine.ny / AMR_RATIO > r.coarse.ny - 1)
            return fail(c, HSGN_EINVAL, "regrid: a new patch leaves its parent");
        r.c0 = ti;
        ti += (long long)r.fine.nx * r.fine.ny;
        I.push_back(r);
        near.clear();
        if (!old_fine.empty()) oidx.near(n->pI0[f], n->pJ0[f], r.fine.nx, r.fine.ny, near);
        for (int &op : near) op = opos[op];
        std::sort(near.begin(), near.end());
        near.erase(std::unique(near.begin(), near.end()), near.end());
        for (int k : near) {
            const int op = old_fine[k];
            const PatchInfo &o = c->patches[op];
            const int ax0 = std::max(n->pI0[f], c->pI0[op]);
            const int ax1 = std::min(n->pI0[f] + r.fine.nx, c->pI0[op] + o.nx);
            const int ay0 = std::max(n->pJ0[f], c->pJ0[op]);
            const int ay1 = std::min(n->pJ0[f] + r.fine.ny, c->pJ0[op] + o.ny);
            if (ax1 <= ax0 || ay1 <= ay0) continue;
            O.push_back(old_rec(op, r.fine, ax0 - c->pI0[op], ay0 - c->pJ0[op], ax0 - n->pI0[f],
                                ay0 - n->pJ0[f], ax1 - ax0, ay1 - ay0, to));
            to += (long long)(ax1 - ax0) * (ay1 - ay0);
        }
    }
    RegridCopy<S> *dK = nullptr, *dO = nullptr;
    RegridInterp *dI = nullptr;
    int rc;
    if ((rc = rg_upload(c, &dK, K)) || (rc = rg_upload(c, &dI, I)) || (rc = rg_upload(c, &dO, O))) {
        if (dK) (void)hipFree(dK);
        if (dI) (void)hipFree(dI);
        if (dO) (void)hipFree(dO);
        return rc;
    }
    const double eta0 = c->prm.eta0, dtol = c->prm.dry_tol;
    if (MIXED) {
        launch_regrid_copy32((const RegridCopy<float> *)dK, (int)K.size(), tk, (float *)nq,
                             (const float *)nb, n->m0, n->m1, eta0, dtol, n->stream);
        launch_regrid_interp32(dI, (int)I.size(), ti, (float *)nq, (const float *)nb, n->m0, n->m1,
                               eta0, dtol, n->stream);
        launch_regrid_copy32((const RegridCopy<float> *)dO, (int)O.size(), to, (float *)nq,
                             (const float *)nb, n->m0, n->m1, eta0, dtol, n->stream);
    } else {
        launch_regrid_copy64((const RegridCopy<double> *)dK, (int)K.size(), tk, (double *)nq,
                             (const double *)nb, n->m0, n->m1, eta0, dtol, n->stream);
        launch_regrid_interp64(dI, (int)I.size(), ti, (double *)nq, (const double *)nb, n->m0,
                               n->m1, eta0, dtol, n->stream);
        launch_regrid_copy64((const RegridCopy<double> *)dO, (int)O.size(), to, (double *)nq,
                             (const double *)nb, n->m0, n->m1, eta0, dtol, n->stream);
    }
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(n->stream);
    if (dK) (void)hipFree(dK);
    if (dI) (void)hipFree(dI);
    if (dO) (void)hipFree(dO);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(c, HSGN_EDEVICE, std::string("regrid transfer: ") +
                                         hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return HSGN_OK;
}

}  // namespace

extern "C" {

int hsgn_num_patches(hsgn_ctx *c, int *n)
{
    if (!c || !n) return HSGN_EINVAL;
    *n = (int)c->patches.size();
    return HSGN_OK;
}

int hsgn_patch_info(hsgn_ctx *c, int patch, int *scenario, int *level, int *nx, int *ny,
                    double *x0, double *y0, double *dx, double *dy)
{
    if (!c || patch < 0 || patch >= (int)c->patches.size())
        return fail(c, HSGN_EINVAL, "bad patch id");
    const PatchInfo &p = c->patches[patch];
    int s = 0;
    for (size_t k = 0; k < c->scen.size(); k++)
        for (int q : c->scen[k].patches)
            if (q == patch) s = (int)k;
    if (scenario) *scenario = s;
    if (level) *level = p.level;
    if (nx) *nx = p.nx;
    if (ny) *ny = p.ny;
    if (x0) *x0 = c->px0[patch];
    if (y0) *y0 = c->py0[patch];
    if (dx) *dx = p.dx;
    if (dy) *dy = p.dy;
    return HSGN_OK;
}

int hsgn_regrid(hsgn_ctx *c, int scenario, const hsgn_regrid_params *r, int *n_new)
{
    if (!c || !c->finalized || !r) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (scenario < 0 || scenario >= (int)c->scen.size())
        return fail(c, HSGN_EINVAL, "bad scenario");
    ScenHost &sh = c->scen[scenario];
    if (!sh.amr) return fail(c, HSGN_ENOTSUP, "regridding needs a patch set (tile level 0)");
    // the rebuilt context carries sponges but not mappings: a mapped single
    // grid beside the patch set would silently become Cartesian
    if (c->any_mapped)
        return fail(c, HSGN_ENOTSUP, "regridding in a context that holds a mapped grid");
    const int level = r->level;
    if (level < 0 || level >= (int)sh.lev.size() || level + 1 > 5 || !(r->tol == r->tol) ||
        r->nbuf < 0 || r->nbuf > 64 || !(r->cutoff > 0.0 && r->cutoff <= 1.0) || r->max_side < 1)
        return fail(c, HSGN_EINVAL, "bad regrid parameters");
    for (int pid : sh.patches) {
        const bool rule = pid < (int)c->braw_rule.size() && c->braw_rule[pid];
        if (!rule && (pid >= (int)c->braw.size() ||
                      c->braw[pid].size() != (size_t)c->patches[pid].nx * c->patches[pid].ny))
            return fail(c, HSGN_EINVAL, "set the bathymetry of every patch before regridding");
    }
    int rc = ensure_prepared(c);
    if (rc) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    // 1-4. flags of the level-l patches, clusters, new level-(l+1) boxes
    struct NewBox { int parent, nx, ny, I0, J0; };
    std::vector<NewBox> boxes;
    std::vector<long long> foff;
    long long ftot = 0;
    for (int pid : sh.lev[level]) {
        foff.push_back(ftot);
        ftot += (long long)c->patches[pid].nx * c->patches[pid].ny;
    }
    // one launch: the patch records, then the flags, in one device buffer
    // (the level-l patches share a clock slot, so one current buffer)
    std::vector<FlagRec> frec(sh.lev[level].size());
    for (size_t k = 0; k < frec.size(); k++) {
        memset(&frec[k], 0, sizeof(FlagRec));
        frec[k].p = c->patches[sh.lev[level][k]];
        frec[k].c0 = foff[k];
    }
    const int cur = frec.empty() ? 0 : st[c->patches[sh.lev[level][0]].scen].cur;
    const size_t rbytes = (sizeof(FlagRec) * frec.size() + 255) / 256 * 256;
    uint8_t *dbuf = nullptr;
    HIPCHK(c, hipMalloc(&dbuf, rbytes + (size_t)std::max<long long>(ftot, 1)));
    const FlagRec *drec = (const FlagRec *)dbuf;
    uint8_t *dflag = dbuf + rbytes;
    std::vector<uint8_t> Fall((size_t)std::max<long long>(ftot, 1));
    hipError_t fe = hipMemcpyAsync(dbuf, frec.data(), sizeof(FlagRec) * frec.size(),
                                   hipMemcpyHostToDevice, c->stream);
    if (fe == hipSuccess) {
        if (c->mixed)
            launch_regrid_flag32(drec, (int)frec.size(), ftot, cur ? c->f1 : c->f0, c->fbath,
                                 dflag, c->prm.eta0, c->prm.dry_tol, r->tol, c->stream);
        else
            launch_regrid_flag64(drec, (int)frec.size(), ftot, cur ? c->q1 : c->q0, c->bath,
                                 dflag, c->prm.eta0, c->prm.dry_tol, r->tol, c->stream);
        fe = hipGetLastError();
    }
    if (fe == hipSuccess)
        fe = hipMemcpyAsync(Fall.data(), dflag, (size_t)ftot, hipMemcpyDeviceToHost, c->stream);
    if (fe == hipSuccess) fe = hipStreamSynchronize(c->stream);
    (void)hipFree(dbuf);
    if (fe != hipSuccess)
        return fail(c, HSGN_EDEVICE, std::string("regrid flags: ") + hipGetErrorString(fe));
    // buffer and clusters per level-l patch, on host threads, joined in
    // patch order
    const size_t np_l = sh.lev[level].size();
    std::vector<std::vector<NewBox>> pboxes(np_l);
    auto cluster_one = [&](size_t k) {
        const int pid = sh.lev[level][k];
        const PatchInfo &p = c->patches[pid];
        const uint8_t *F = Fall.data() + foff[k];
        // the buffer: flags dilated by nbuf cells in the max norm (within the
        // patch), as a pass along rows and one along columns, each counting
        // the flags in its sliding window
        const int nx = p.nx, ny = p.ny, nb = r->nbuf;
        std::vector<uint8_t> R((size_t)nx * ny), B((size_t)nx * ny);
        for (int j = 0; j < ny; j++) {
            const uint8_t *f = F + (size_t)j * nx;
            int cnt = 0;
            for (int a = 0; a < std::min(nb, nx); a++) cnt += f[a] != 0;
            for (int i = 0; i < nx; i++) {
                if (i + nb < nx) cnt += f[i + nb] != 0;
                if (i - nb - 1 >= 0) cnt -= f[i - nb - 1] != 0;
                R[(size_t)j * nx + i] = cnt > 0;
            }
        }
        std::vector<int> col(nx, 0);
        for (int b = 0; b < std::min(nb, ny); b++)
            for (int i = 0; i < nx; i++) col[i] += R[(size_t)b * nx + i];
        for (int j = 0; j < ny; j++) {
            if (j + nb < ny)
                for (int i = 0; i < nx; i++) col[i] += R[(size_t)(j + nb) * nx + i];
            if (j - nb - 1 >= 0)
                for (int i = 0; i < nx; i++) col[i] -= R[(size_t)(j - nb - 1) * nx + i];
            for (int i = 0; i < nx; i++) B[(size_t)j * nx + i] = col[i] > 0;
        }
        std::vector<RgBox> cl;
        rg_cluster(B, p.nx, 0, p.nx, 0, p.ny, r->cutoff, r->max_side, cl);
        for (const RgBox &x : cl) {
            const int i0 = std::max(x.i0, 1), i1 = std::min(x.i1, p.nx - 1);
            const int j0 = std::max(x.j0, 1), j1 = std::min(x.j1, p.ny - 1);
            if (i1 <= i0 || j1 <= j0) continue;
            pboxes[k].push_back({pid, AMR_RATIO * (i1 - i0), AMR_RATIO * (j1 - j0),
                                 AMR_RATIO * (c->pI0[pid] + i0), AMR_RATIO * (c->pJ0[pid] + j0)});
        }
    };
    // one task per patch (the flags and so the clustering work differ)
    if (np_l > 8)
        HostPool::get().parallel_for((int)np_l, [&](int k) { cluster_one((size_t)k); });
    else
        for (size_t k = 0; k < np_l; k++) cluster_one(k);
    for (auto &v : pboxes) boxes.insert(boxes.end(), v.begin(), v.end());
    // 5. the new context: every patch of the other scenarios, the levels <= l
    // of this one, then the new boxes
    hsgn_ctx *n = nullptr;
    if ((rc = hsgn_create(&c->prm, c->stream, &n))) return fail(c, rc, "regrid: context");
    auto bail = [&](int code, const std::string &why) {
        std::string msg = why + (n->last_error.empty() ? "" : ": " + n->last_error);
        hsgn_destroy(n);
        return fail(c, code, msg);
    };
    std::vector<int> newid(c->patches.size(), -1);
    std::vector<std::pair<int, int>> kept, fresh;     // (old, new); (new, new parent)
    std::vector<int> old_fine;
    double dx0 = 0.0, dy0 = 0.0;
    for (size_t s = 0; s < c->scen.size(); s++)
        for (int pid : c->scen[s].patches) {
            const PatchInfo &p = c->patches[pid];
            if ((int)s == scenario && p.level > level) {
                if (p.level == level + 1) old_fine.push_back(pid);
                continue;
            }
            if ((int)s == scenario && p.level == 0) { dx0 = p.dx; dy0 = p.dy; }
            int id = -1;
            if ((rc = hsgn_add_grid(n, (int)s, p.level, p.nx, p.ny, c->px0[pid], c->py0[pid],
                                    p.dx, p.dy, p.bc, &id)))
                return bail(rc, "regrid: add_grid");
            newid[pid] = id;
            kept.push_back({pid, id});
        }
    const double sc = (double)(1LL << (2 * (level + 1)));
    const double dxf = dx0 / sc, dyf = dy0 / sc;
    const int *bc0 = c->patches[sh.lev[0][0]].bc;
    std::vector<int> fresh_ids;
    for (const NewBox &b : boxes) {
        int id = -1;
        if ((rc = hsgn_add_grid(n, scenario, level + 1, b.nx, b.ny, sh.X0 + b.I0 * dxf,
                                sh.Y0 + b.J0 * dyf, dxf, dyf, bc0, &id)))
            return bail(rc, "regrid: add_grid (new patch)");
        fresh.push_back({id, newid[b.parent]});
        fresh_ids.push_back(id);
    }
    // the old context's host tables lend their memory to the new context's
    // (the old one keeps its device tables and record counts)
    n->h_gc.swap(c->h_gc);
    n->h_gi.swap(c->h_gi);
    n->h_fr.swap(c->h_fr);
    n->h_av.swap(c->h_av);
    if ((rc = hsgn_finalize(n))) return bail(rc, "regrid: finalize");
    n->timing = c->timing;
    for (size_t s = 0; s < c->scen.size() && s < n->scen.size(); s++) {
        if (!(c->scen[s].sp_rate > 0.0)) continue;
        for (int e = 0; e < 4; e++) n->scen[s].sp_w[e] = c->scen[s].sp_w[e];
        n->scen[s].sp_rate = c->scen[s].sp_rate;
        n->any_sponge = true;
        if ((rc = apply_sponge(n, (int)s))) return bail(rc, "regrid: sponge");
    }
    // bathymetry: level-0 and regridded patches from the level-0 bathymetry
    // B0 (on the device; at level 0 the rule returns B0 itself), patches given
    // by the caller from their host copies (one transfer)
    n->braw.assign(n->patches.size(), std::vector<double>());
    n->braw_rule.assign(n->patches.size(), 0);
    // host bathymetry copies carried over: moved once the regrid has succeeded
    std::vector<int> braw_src(n->patches.size(), -1);
    {
        // the level-0 bathymetry on the device, kept for the next regrid of
        // this scenario until a bathymetry changes
        const bool b0_cached = c->d_B0 && c->b0_scen == scenario;
        std::vector<double> B0;
        if (!b0_cached) {
            B0.resize((size_t)sh.NX * sh.NY);
            for (int pid : sh.lev[0]) {
                const PatchInfo &p = c->patches[pid];
                for (int j = 0; j < p.ny; j++)
                    memcpy(&B0[(size_t)(c->pJ0[pid] + j) * sh.NX + c->pI0[pid]],
                           &c->braw[pid][(size_t)j * p.nx], sizeof(double) * p.nx);
            }
        }
        std::vector<TopoRec> topo;
        std::vector<BulkRec> bulk;
        long long ttot = 0, btot = 0;
        auto add_topo = [&](int id) {
            TopoRec t;
            memset(&t, 0, sizeof(t));
            t.p = n->patches[id];
            t.I0 = n->pI0[id]; t.J0 = n->pJ0[id]; t.level = n->patches[id].level;
            t.c0 = ttot;
            ttot += (long long)t.p.nx * t.p.ny;
            topo.push_back(t);
        };
        for (auto &k : kept) {
            const bool this_scen = n->slot_scen[n->patches[k.second].scen] == scenario;
            const bool rule = k.first < (int)c->braw_rule.size() && c->braw_rule[k.first];
            if (this_scen && (c->patches[k.first].level == 0 || rule)) {
                add_topo(k.second);
                n->braw_rule[k.second] = rule ? 1 : 0;
                if (!rule) braw_src[k.second] = k.first;
            } else if (rule) {
                return bail(HSGN_EINVAL, "regrid: rule bathymetry outside its scenario");
            } else {
                braw_src[k.second] = k.first;
                bulk.push_back({n->patches[k.second], btot});
                btot += (long long)c->braw[k.first].size();
            }
        }
        for (int id : fresh_ids) {
            add_topo(id);
            n->braw_rule[id] = 1;
        }
        std::vector<double> all((size_t)std::max<long long>(btot, 1));
        for (size_t k = 0, pos = 0; k < kept.size(); k++) {
            const int id = kept[k].second;
            if (braw_src[id] < 0 || n->braw_rule[id]) continue;
            const bool topo_done = n->slot_scen[n->patches[id].scen] == scenario &&
                                   n->patches[id].level == 0;
            if (topo_done) continue;
            const std::vector<double> &src = c->braw[braw_src[id]];
            memcpy(&all[pos], src.data(), sizeof(double) * src.size());
            pos += src.size();
        }
        double *dB0 = b0_cached ? c->d_B0 : nullptr, *din = nullptr;
        TopoRec *dtopo = nullptr;
        BulkRec *dbulk = nullptr;
        hipError_t be = hipSuccess;
        if (!b0_cached) {
            be = hipMalloc(&dB0, sizeof(double) * B0.size());
            if (be == hipSuccess) n->d_B0 = dB0;            // the new context owns it
            if (be == hipSuccess)
                be = hipMemcpy(dB0, B0.data(), sizeof(double) * B0.size(), hipMemcpyHostToDevice);
        }
        n->b0_scen = scenario;
        if (be == hipSuccess && !topo.empty()) {
            be = hipMalloc(&dtopo, sizeof(TopoRec) * topo.size());
            if (be == hipSuccess)
                be = hipMemcpy(dtopo, topo.data(), sizeof(TopoRec) * topo.size(), hipMemcpyHostToDevice);
        }
        if (be == hipSuccess && !bulk.empty()) {
            be = hipMalloc(&din, sizeof(double) * btot);
            if (be == hipSuccess) be = hipMalloc(&dbulk, sizeof(BulkRec) * bulk.size());
            if (be == hipSuccess)
                be = hipMemcpy(din, all.data(), sizeof(double) * btot, hipMemcpyHostToDevice);
            if (be == hipSuccess)
                be = hipMemcpy(dbulk, bulk.data(), sizeof(BulkRec) * bulk.size(), hipMemcpyHostToDevice);
        }
        if (be == hipSuccess) {
            if (n->mixed) {
                launch_topo32(dtopo, (int)topo.size(), ttot, dB0, sh.NX, sh.NY, n->fbath, n->stream);
                if (!bulk.empty())
                    scatter_bulk_kernel<float><<<nblk(btot), 256, 0, n->stream>>>(
                        dbulk, (int)bulk.size(), btot, din, n->fbath);
            } else {
                launch_topo64(dtopo, (int)topo.size(), ttot, dB0, sh.NX, sh.NY, n->bath, n->stream);
                if (!bulk.empty())
                    scatter_bulk_kernel<double><<<nblk(btot), 256, 0, n->stream>>>(
                        dbulk, (int)bulk.size(), btot, din, n->bath);
            }
            // single grids: phi_T from their bathymetry (patch sets: at preparation)
            for (size_t pid = 0; pid < n->patches.size(); pid++) {
                const PatchInfo &p = n->patches[pid];
                if (p.frame) continue;
                unsigned nb = nblk((long long)p.nx * p.ny);
                if (n->mixed)
                    mask_kernel<float><<<nb, 256, 0, n->stream>>>(p, n->fbath, n->m0, n->m1,
                                                                  n->prm.eta0, n->prm.h_star,
                                                                  n->prm.nbr_n);
                else
                    mask_kernel<double><<<nb, 256, 0, n->stream>>>(p, n->bath, n->m0, n->m1,
                                                                   n->prm.eta0, n->prm.h_star,
                                                                   n->prm.nbr_n);
            }
            be = hipGetLastError();
            if (be == hipSuccess) be = hipStreamSynchronize(n->stream);
        }
        if (dtopo) (void)hipFree(dtopo);
        if (din) (void)hipFree(din);
        if (dbulk) (void)hipFree(dbulk);
        if (be != hipSuccess)
            return bail(HSGN_EDEVICE, std::string("regrid: bathymetry: ") + hipGetErrorString(be));
        n->amr_dirty = n->any_amr;
    }
    if ((rc = ensure_prepared(n))) return bail(rc, "regrid: prepare");
    // 6. the state
    for (auto &f : fresh) {
        if (n->pI0[f.first] % AMR_RATIO || n->pJ0[f.first] % AMR_RATIO)
            return bail(HSGN_EINVAL, "regrid: misaligned patch");
    }
    rc = c->mixed ? rg_transfer<float, true>(c, n, st, kept, fresh, old_fine, level)
                  : rg_transfer<double, false>(c, n, st, kept, fresh, old_fine, level);
    if (rc) { hsgn_destroy(n); return rc; }
    n->state_set.assign(n->patches.size(), 1);    // every patch's state was moved in
    // 7. clocks, clipped mass, gauges and their records
    std::vector<ScenState> sn;
    if ((rc = pull_scen(n, sn))) return bail(rc, "regrid: clock");
    std::vector<std::vector<double>> recs(c->scen.size());
    std::vector<long long> nrec(c->scen.size(), 0);
    for (size_t s = 0; s < c->scen.size(); s++) {
        const ScenHost &o = c->scen[s];
        const ScenState &o0 = st[o.slot[0]];
        double clip = 0.0;
        for (int sl : o.slot) clip += st[sl].clip_total;
        if (!c->h_rf.empty()) {
            std::vector<double> rcl(c->h_rf.size());
            HIPCHK(c, hipMemcpy(rcl.data(), c->d_rclip, sizeof(double) * rcl.size(),
                                hipMemcpyDeviceToHost));
            for (size_t k = 0; k < rcl.size(); k++)
                for (int sl : o.slot)
                    if (c->patches[c->h_rf[k].cp].scen == sl) clip += rcl[k];
        }
        const ScenHost &nh = n->scen[s];
        long long f = 1;
        for (size_t l = 0; l < nh.slot.size(); l++) {
            ScenState &x = sn[nh.slot[l]];
            const ScenState *src = l < o.slot.size() ? &st[o.slot[l]] : &o0;
            x = *src;
            x.cur = 0;
            x.records = 0;
            x.clip_total = l == 0 ? clip : 0.0;
            if (l >= o.slot.size()) {
                x.t = o0.t;
                x.dt = o0.dt / (double)f;
                x.dt_fixed = o0.dt_fixed / (double)f;
                x.steps = o0.steps * f;
                x.max_courant = 0.0;
            }
            f *= AMR_RATIO;
        }
        // gauge records not yet read
        nrec[s] = std::min<long long>(o0.records, o.gcap);
        if (o.ng > 0 && nrec[s] > 0 && c->rec) {
            recs[s].resize((size_t)nrec[s] * (1 + o.ng));
            HIPCHK(c, hipMemcpy(recs[s].data(), c->rec + o.roff, sizeof(double) * recs[s].size(),
                                hipMemcpyDeviceToHost));
        }
    }
    if ((rc = push_scen(n, sn))) return bail(rc, "regrid: clock");
    for (size_t s = 0; s < c->scen.size(); s++)
        if (c->scen[s].ng > 0 &&
            (rc = hsgn_set_gauges(n, (int)s, c->scen[s].ng, c->scen[s].gauge_xy.data())))
            return bail(rc, "regrid: gauges");
    if ((rc = pull_scen(n, sn))) return bail(rc, "regrid: clock");
    for (size_t s = 0; s < c->scen.size(); s++) sn[s].records = nrec[s];
    if ((rc = ensure_gauges(n, sn, 0))) return bail(rc, "regrid: gauge records");
    for (size_t s = 0; s < c->scen.size(); s++)
        if (!recs[s].empty()) {
            hipError_t e = hipMemcpy(n->rec + n->scen[s].roff, recs[s].data(),
                                     sizeof(double) * recs[s].size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return bail(HSGN_EDEVICE, "regrid: gauge records");
        }
    if ((rc = push_scen(n, sn))) return bail(rc, "regrid: clock");
    // 8. the new context replaces the old one (with the kernel timing so far)
    if ((rc = collect_timing(c))) return bail(rc, "regrid: timing");
    n->timed_ms = c->timed_ms;
    n->timed_launches = c->timed_launches;
    // hand-over of what the new context takes from the old one
    if (!n->d_B0 && c->b0_scen == scenario) {
        n->d_B0 = c->d_B0;
        c->d_B0 = nullptr;
    }
    for (size_t id = 0; id < braw_src.size(); id++)
        if (braw_src[id] >= 0) n->braw[id] = std::move(c->braw[braw_src[id]]);
    std::swap(*c, *n);
    hsgn_destroy(n);
    if (n_new) *n_new = (int)boxes.size();
    return HSGN_OK;
}

}  // extern "C"
