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
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hsgn.h"
#include "hsgn_march.hpp"

using namespace hsgn;

// ---------------------------------------------------------------------------
// device side

// the step kernel is compiled in two translation units with different
// floating-point contraction (hsgn_step64.hip: none, hsgn_step32.hip: FMA)
void launch_march64(const MarchArgs<double> &A, unsigned nwork, hipStream_t stream);
void launch_march32(const MarchArgs<float> &A, unsigned nwork, hipStream_t stream);

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
    int pad;
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
    const S *q = st.cur ? q1 : q0;
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
            int mx = map_index(x + di, pi.nx, pi.bc[0], pi.bc[1], &fx);
            int my = map_index(y + dj, pi.ny, pi.bc[2], pi.bc[3], &fy);
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
        long long plane = (long long)pi.ny * pi.pitch;
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
            double c2 = swe ? 0.0 : P.a2g * H;
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

// FP64 sum of h over one patch: fixed decomposition (1024 threads, strided),
// then a fixed-order tree in shared memory
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

// conversion between the ABI layout (FP64, plane 0 = h) and FP32 storage
// (plane 0 = eta' = h + b - eta0)
__global__ void to_storage_kernel(PatchInfo pi, const double *in, float *q, const float *bath,
                                  double eta0)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    long long idx = (long long)y * pi.pitch + x;
    long long plane = (long long)pi.ny * pi.pitch;
    double b = (double)bath[pi.coff + idx];
    q[pi.qoff + idx] = (float)(in[i] + b - eta0);
    for (int m = 1; m < 7; m++) q[pi.qoff + m * plane + idx] = (float)in[m * ncell + i];
}

__global__ void from_storage_kernel(PatchInfo pi, const float *q, const float *bath, double eta0,
                                    double *out)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long ncell = (long long)pi.nx * pi.ny;
    if (i >= ncell) return;
    int x = (int)(i % pi.nx), y = (int)(i / pi.nx);
    long long idx = (long long)y * pi.pitch + x;
    long long plane = (long long)pi.ny * pi.pitch;
    double b = (double)bath[pi.coff + idx];
    double h = (double)q[pi.qoff + idx] + eta0 - b;
    out[i] = h > 0.0 ? h : 0.0;
    for (int m = 1; m < 7; m++) out[m * ncell + i] = (double)q[pi.qoff + m * plane + idx];
}

__global__ void to_float_kernel(const double *in, float *out, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// host side

struct ScenHost {
    std::vector<int> patches;
    std::vector<double> gauge_xy;
    long long gcap = 0, roff = 0;
    int ng = 0;
};

struct hsgn_ctx {
    hsgn_params prm;
    StepParams P;
    hipStream_t stream = nullptr;
    bool finalized = false;
    std::vector<PatchInfo> patches;
    std::vector<double> px0, py0;
    std::vector<ScenHost> scen;
    std::vector<WorkItem> work;
    std::vector<ScenStatic> sstat;
    bool mixed = false;         // FP32 eta' storage with FP64 near-shore edges
    // device (FP64 storage: q0, q1, bath; mixed storage: f0, f1, fbath)
    double *q0 = nullptr, *q1 = nullptr, *bath = nullptr, *clip = nullptr, *rec = nullptr;
    float *f0 = nullptr, *f1 = nullptr, *fbath = nullptr;
    double *stage = nullptr;    // FP64 staging for conversions at the ABI
    long long stage_len = 0;
    uint8_t *m0 = nullptr, *m1 = nullptr;
    PatchInfo *d_patches = nullptr;
    WorkItem *d_work = nullptr;
    ScenState *d_scen = nullptr;
    ScenStatic *d_sstat = nullptr;
    GaugeDev *d_gauges = nullptr;
    unsigned long long *d_slots = nullptr;
    int *d_err = nullptr;
    double *d_mass = nullptr;
    int ngauge_total = 0;
    long long qtotal = 0, ctotal = 0, rec_total = 0;
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

static void free_device(hsgn_ctx *c)
{
    free_events(c);
    void *ptrs[] = {c->q0, c->q1, c->bath, c->clip, c->rec, c->m0, c->m1, c->d_patches,
                    c->d_work, c->d_scen, c->d_sstat, c->d_gauges, c->d_slots, c->d_err,
                    c->d_mass, c->f0, c->f1, c->fbath, c->stage};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    c->q0 = c->q1 = c->bath = c->clip = c->rec = c->d_mass = c->stage = nullptr;
    c->f0 = c->f1 = c->fbath = nullptr;
    c->m0 = c->m1 = nullptr;
    c->d_patches = nullptr; c->d_work = nullptr; c->d_scen = nullptr; c->d_sstat = nullptr;
    c->d_gauges = nullptr; c->d_slots = nullptr; c->d_err = nullptr;
}

template <class S>
static MarchArgs<S> march_args(hsgn_ctx *c, S *q0, S *q1, const S *bath)
{
    MarchArgs<S> A;
    A.P = c->P;
    A.patches = c->d_patches;
    A.work = c->d_work;
    A.q0 = q0; A.q1 = q1;
    A.bath = bath;
    A.m0 = c->m0; A.m1 = c->m1;
    A.scen = c->d_scen;
    A.clip_slots = c->clip;
    A.nwork = (int)c->work.size();
    return A;
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
    default: return "unknown status";
    }
}

const char *hsgn_last_error(hsgn_ctx *c) { return c ? c->last_error.c_str() : ""; }

int hsgn_create(const hsgn_params *p, void *hip_stream, hsgn_ctx **out)
{
    if (!p || !out) return HSGN_EINVAL;
    *out = nullptr;
    if (p->model != 0 || (p->precision != 0 && p->precision != 1)) return HSGN_ENOTSUP;
    if (!(p->g > 0) || p->alpha < 0 || !(p->dry_tol >= 0) || !(p->cfl > 0) ||
        !(p->cfl_max >= p->cfl) || p->nbr_n < 0 || p->nbr_n > 2 || p->limiter < 0 ||
        p->limiter > 3 || (p->transverse != 0 && p->transverse != 2) ||
        (p->splitting != 0 && p->splitting != 1) || !(p->xi1 > 0))
        return HSGN_EINVAL;
    hsgn_ctx *c = new (std::nothrow) hsgn_ctx();
    if (!c) return HSGN_ENOMEM;
    c->prm = *p;
    c->mixed = p->precision == 1;
    c->stream = (hipStream_t)hip_stream;
    StepParams &P = c->P;
    P.g = p->g;
    P.a2g = p->alpha * p->alpha * p->g;
    P.eta0 = p->eta0; P.h_star = p->h_star; P.dry_tol = p->dry_tol;
    P.xi0 = p->xi0; P.xi1 = p->xi1; P.kappa = p->kappa;
    P.limiter = p->limiter; P.transverse = p->transverse; P.splitting = p->splitting;
    *out = c;
    return HSGN_OK;
}

int hsgn_add_grid(hsgn_ctx *c, int scenario, int nx, int ny, double x0, double y0, double dx,
                  double dy, const int bc[4], int *patch_id)
{
    if (!c) return HSGN_EINVAL;
    if (c->finalized) return fail(c, HSGN_EINVAL, "add_grid after finalize");
    if (scenario < 0 || nx < 4 || ny < 4 || !(dx > 0) || !(dy > 0) || !bc)
        return fail(c, HSGN_EINVAL, "bad grid arguments");
    for (int k = 0; k < 4; k++)
        if (bc[k] < 0 || bc[k] > 2) return fail(c, HSGN_EINVAL, "bad boundary condition");
    if ((bc[0] == HSGN_BC_PERIODIC) != (bc[1] == HSGN_BC_PERIODIC) ||
        (bc[2] == HSGN_BC_PERIODIC) != (bc[3] == HSGN_BC_PERIODIC))
        return fail(c, HSGN_EINVAL, "periodic sides must come in pairs");
    if ((int)c->scen.size() <= scenario) c->scen.resize(scenario + 1);
    if (!c->scen[scenario].patches.empty()) {
        const PatchInfo &f = c->patches[c->scen[scenario].patches[0]];
        if (f.dx != dx || f.dy != dy)
            return fail(c, HSGN_EINVAL, "patches of one scenario share dx, dy");
    }
    PatchInfo pi;
    memset(&pi, 0, sizeof(pi));
    pi.nx = nx; pi.ny = ny; pi.pitch = nx; pi.scen = scenario;
    for (int k = 0; k < 4; k++) pi.bc[k] = bc[k];
    pi.dx = dx; pi.dy = dy;
    c->patches.push_back(pi);
    c->px0.push_back(x0);
    c->py0.push_back(y0);
    int id = (int)c->patches.size() - 1;
    c->scen[scenario].patches.push_back(id);
    if (patch_id) *patch_id = id;
    return HSGN_OK;
}

static int choose_rows(const hsgn_ctx *c)
{
    if (c->prm.tile_rows > 0) return c->prm.tile_rows;
    // enough wavefronts to fill the chip several times over: 256 CUs x 4 SIMDs
    long long cells = 0;
    for (const PatchInfo &p : c->patches) cells += (long long)p.nx * p.ny;
    long long target_waves = 4096;
    long long cells_per_wave = std::max<long long>(60 * 8, cells / target_waves);
    int th = (int)std::min<long long>(64, std::max<long long>(8, cells_per_wave / 60));
    return th;
}

int hsgn_finalize(hsgn_ctx *c)
{
    if (!c) return HSGN_EINVAL;
    if (c->finalized) return fail(c, HSGN_EINVAL, "finalize called twice");
    if (c->patches.empty()) return fail(c, HSGN_EINVAL, "no patches");
    for (size_t s = 0; s < c->scen.size(); s++)
        if (c->scen[s].patches.empty()) return fail(c, HSGN_EINVAL, "scenario numbers must be dense");
    long long qo = 0, co = 0;
    for (PatchInfo &p : c->patches) {
        long long cells = (long long)p.pitch * p.ny;
        p.qoff = qo;
        p.coff = co;
        qo += 7 * cells;
        co += cells;
    }
    c->qtotal = qo;
    c->ctotal = co;
    int th = choose_rows(c);
    c->work.clear();
    c->sstat.assign(c->scen.size(), ScenStatic());
    for (size_t s = 0; s < c->scen.size(); s++) {
        ScenStatic &ss = c->sstat[s];
        ss.dx = c->patches[c->scen[s].patches[0]].dx;
        ss.dy = c->patches[c->scen[s].patches[0]].dy;
        ss.cfl = c->prm.cfl;
        ss.cfl_max = c->prm.cfl_max;
        ss.w0 = (int)c->work.size();
        for (int pid : c->scen[s].patches) {
            const PatchInfo &p = c->patches[pid];
            for (int r0 = 0; r0 < p.ny; r0 += th)
                for (int i0 = 0; i0 < p.nx; i0 += 60)
                    c->work.push_back({pid, i0, r0, std::min(th, p.ny - r0)});
        }
        ss.w1 = (int)c->work.size();
    }
    size_t nscen = c->scen.size();
    if (c->mixed) {
        HIPCHK(c, hipMalloc(&c->f0, sizeof(float) * c->qtotal));
        HIPCHK(c, hipMalloc(&c->f1, sizeof(float) * c->qtotal));
        HIPCHK(c, hipMalloc(&c->fbath, sizeof(float) * c->ctotal));
        HIPCHK(c, hipMemsetAsync(c->f0, 0, sizeof(float) * c->qtotal, c->stream));
        HIPCHK(c, hipMemsetAsync(c->f1, 0, sizeof(float) * c->qtotal, c->stream));
        HIPCHK(c, hipMemsetAsync(c->fbath, 0, sizeof(float) * c->ctotal, c->stream));
        long long big = 0;
        for (const PatchInfo &p : c->patches) big = std::max<long long>(big, 7LL * p.nx * p.ny);
        c->stage_len = big;
        HIPCHK(c, hipMalloc(&c->stage, sizeof(double) * big));
    } else {
        HIPCHK(c, hipMalloc(&c->q0, sizeof(double) * c->qtotal));
        HIPCHK(c, hipMalloc(&c->q1, sizeof(double) * c->qtotal));
        HIPCHK(c, hipMalloc(&c->bath, sizeof(double) * c->ctotal));
        HIPCHK(c, hipMemsetAsync(c->q0, 0, sizeof(double) * c->qtotal, c->stream));
        HIPCHK(c, hipMemsetAsync(c->q1, 0, sizeof(double) * c->qtotal, c->stream));
        HIPCHK(c, hipMemsetAsync(c->bath, 0, sizeof(double) * c->ctotal, c->stream));
    }
    HIPCHK(c, hipMalloc(&c->m0, c->ctotal));
    HIPCHK(c, hipMalloc(&c->m1, c->ctotal));
    HIPCHK(c, hipMalloc(&c->clip, sizeof(double) * c->work.size()));
    HIPCHK(c, hipMalloc(&c->d_patches, sizeof(PatchInfo) * c->patches.size()));
    HIPCHK(c, hipMalloc(&c->d_work, sizeof(WorkItem) * c->work.size()));
    HIPCHK(c, hipMalloc(&c->d_scen, sizeof(ScenState) * nscen));
    HIPCHK(c, hipMalloc(&c->d_sstat, sizeof(ScenStatic) * nscen));
    HIPCHK(c, hipMalloc(&c->d_slots, sizeof(unsigned long long) * nscen));
    HIPCHK(c, hipMalloc(&c->d_err, sizeof(int)));
    HIPCHK(c, hipMalloc(&c->d_mass, sizeof(double) * 2));
    HIPCHK(c, hipMemsetAsync(c->m0, 0, c->ctotal, c->stream));
    HIPCHK(c, hipMemsetAsync(c->m1, 0, c->ctotal, c->stream));
    HIPCHK(c, hipMemsetAsync(c->clip, 0, sizeof(double) * c->work.size(), c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_patches, c->patches.data(), sizeof(PatchInfo) * c->patches.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_work, c->work.data(), sizeof(WorkItem) * c->work.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_sstat, c->sstat.data(), sizeof(ScenStatic) * nscen,
                             hipMemcpyHostToDevice, c->stream));
    std::vector<ScenState> st(nscen);
    memset(st.data(), 0, sizeof(ScenState) * nscen);
    HIPCHK(c, hipMemcpyAsync(c->d_scen, st.data(), sizeof(ScenState) * nscen,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->finalized = true;
    return HSGN_OK;
}

static int pull_scen(hsgn_ctx *c, std::vector<ScenState> &st)
{
    st.resize(c->scen.size());
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

int hsgn_set_bathymetry(hsgn_ctx *c, int patch, const double *b, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!b) return fail(c, HSGN_EINVAL, "null bathymetry");
    const PatchInfo &p = c->patches[patch];
    long long n = (long long)p.nx * p.ny;
    unsigned nb = (unsigned)((n + 255) / 256);
    if (c->mixed) {
        // stored in FP32; phi_T is computed from the stored values
        HIPCHK(c, hipMemcpyAsync(c->stage, b, sizeof(double) * n, kind_in(on_device), c->stream));
        to_float_kernel<<<nb, 256, 0, c->stream>>>(c->stage, c->fbath + p.coff, n);
        mask_kernel<float><<<nb, 256, 0, c->stream>>>(p, c->fbath, c->m0, c->m1, c->prm.eta0,
                                                      c->prm.h_star, c->prm.nbr_n);
    } else {
        HIPCHK(c, hipMemcpyAsync(c->bath + p.coff, b, sizeof(double) * n, kind_in(on_device),
                                 c->stream));
        mask_kernel<double><<<nb, 256, 0, c->stream>>>(p, c->bath, c->m0, c->m1, c->prm.eta0,
                                                       c->prm.h_star, c->prm.nbr_n);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_set_state(hsgn_ctx *c, int patch, const double *q, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!q) return fail(c, HSGN_EINVAL, "null state");
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    const PatchInfo &p = c->patches[patch];
    if (c->mixed) {
        long long n = (long long)p.nx * p.ny;
        HIPCHK(c, hipMemcpyAsync(c->stage, q, sizeof(double) * 7 * n, kind_in(on_device), c->stream));
        float *dst = st[p.scen].cur ? c->f1 : c->f0;
        to_storage_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
            p, c->stage, dst, c->fbath, c->prm.eta0);
        HIPCHK(c, hipGetLastError());
    } else {
        double *dst = (st[p.scen].cur ? c->q1 : c->q0) + p.qoff;
        HIPCHK(c, hipMemcpyAsync(dst, q, sizeof(double) * 7 * p.nx * p.ny, kind_in(on_device),
                                 c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_get_state(hsgn_ctx *c, int patch, double *q, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    if (!q) return fail(c, HSGN_EINVAL, "null output");
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    const PatchInfo &p = c->patches[patch];
    if (c->mixed) {
        long long n = (long long)p.nx * p.ny;
        const float *src = st[p.scen].cur ? c->f1 : c->f0;
        from_storage_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
            p, src, c->fbath, c->prm.eta0, c->stage);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(q, c->stage, sizeof(double) * 7 * n, kind_out(on_device), c->stream));
    } else {
        const double *src = (st[p.scen].cur ? c->q1 : c->q0) + p.qoff;
        HIPCHK(c, hipMemcpyAsync(q, src, sizeof(double) * 7 * p.nx * p.ny, kind_out(on_device),
                                 c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_get_mask(hsgn_ctx *c, int patch, uint8_t *m, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    std::vector<ScenState> st;
    if ((rc = pull_scen(c, st))) return rc;
    const PatchInfo &p = c->patches[patch];
    const uint8_t *src = (st[p.scen].cur ? c->m1 : c->m0) + p.coff;
    HIPCHK(c, hipMemcpyAsync(m, src, (size_t)p.nx * p.ny, kind_out(on_device), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_set_mask(hsgn_ctx *c, int patch, const uint8_t *m, int on_device)
{
    int rc = check_patch(c, patch);
    if (rc) return rc;
    const PatchInfo &p = c->patches[patch];
    HIPCHK(c, hipMemcpyAsync(c->m0 + p.coff, m, (size_t)p.nx * p.ny, kind_in(on_device), c->stream));
    HIPCHK(c, hipMemcpyAsync(c->m1 + p.coff, m, (size_t)p.nx * p.ny, kind_in(on_device), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HSGN_OK;
}

int hsgn_set_gauges(hsgn_ctx *c, int scenario, int n, const double *xy)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (scenario < 0 || scenario >= (int)c->scen.size() || n < 0 || (n > 0 && !xy))
        return fail(c, HSGN_EINVAL, "bad gauge arguments");
    for (int k = 0; k < n; k++) {
        bool found = false;
        for (int pid : c->scen[scenario].patches) {
            const PatchInfo &p = c->patches[pid];
            double x = xy[2 * k], y = xy[2 * k + 1];
            if (x >= c->px0[pid] && x <= c->px0[pid] + p.nx * p.dx && y >= c->py0[pid] &&
                y <= c->py0[pid] + p.ny * p.dy) { found = true; break; }
        }
        if (!found) return fail(c, HSGN_ERANGE, "gauge outside the scenario");
    }
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
            int pid = -1;
            for (int q : sh.patches) {
                const PatchInfo &p = c->patches[q];
                if (x >= c->px0[q] && x <= c->px0[q] + p.nx * p.dx && y >= c->py0[q] &&
                    y <= c->py0[q] + p.ny * p.dy) { pid = q; break; }
            }
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
    if (c->d_gauges) { (void)hipFree(c->d_gauges); c->d_gauges = nullptr; }
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

static int launch_attempt(hsgn_ctx *c)
{
    if (c->timing) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int k = 0; k < 256; k++) {
                hipEvent_t e;
                HIPCHK(c, hipEventCreate(&e));
                c->ev.push_back(e);
            }
        }
        HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
    }
    unsigned nw = (unsigned)c->work.size();
    if (c->mixed)
        launch_march32(march_args<float>(c, c->f0, c->f1, c->fbath), nw, c->stream);
    else
        launch_march64(march_args<double>(c, c->q0, c->q1, c->bath), nw, c->stream);
    if (c->timing) {
        HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
        c->ev_used += 2;
    }
    int ns = (int)c->scen.size();
    control_kernel<<<(unsigned)ns, 256, 0, c->stream>>>(c->d_scen, c->d_sstat, c->clip, ns);
    if (c->ngauge_total > 0) {
        unsigned gb = (unsigned)((c->ngauge_total + 63) / 64);
        if (c->mixed)
            gauge_kernel<float, true><<<gb, 64, 0, c->stream>>>(
                c->d_gauges, c->ngauge_total, c->d_scen, c->f0, c->f1, c->fbath, c->prm.eta0,
                c->prm.dry_tol, c->rec);
        else
            gauge_kernel<double, false><<<gb, 64, 0, c->stream>>>(
                c->d_gauges, c->ngauge_total, c->d_scen, c->q0, c->q1, c->bath, c->prm.eta0,
                c->prm.dry_tol, c->rec);
    }
    HIPCHK(c, hipGetLastError());
    return HSGN_OK;
}

int hsgn_advance(hsgn_ctx *c, double dt, int n_steps)
{
    if (!c || !c->finalized) return fail(c, HSGN_EINVAL, "call hsgn_finalize first");
    if (n_steps < 0) return fail(c, HSGN_EINVAL, "negative step count");
    if (n_steps == 0) return HSGN_OK;
    std::vector<ScenState> st;
    int rc = pull_scen(c, st);
    if (rc) return rc;
    // dt > 0: one fixed step for all scenarios; dt == 0: adaptive steps;
    // dt < 0: each scenario keeps the fixed step stored in its clock
    bool adaptive = dt == 0.0;
    bool per_scen = dt < 0.0;
    bool need_dt0 = false;
    for (size_t s = 0; s < st.size(); s++) {
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
    }
    if ((rc = push_scen(c, st))) return rc;
    if (need_dt0) {
        int ns = (int)c->scen.size();
        HIPCHK(c, hipMemsetAsync(c->d_slots, 0, sizeof(unsigned long long) * ns, c->stream));
        HIPCHK(c, hipMemsetAsync(c->d_err, 0, sizeof(int), c->stream));
        for (size_t pid = 0; pid < c->patches.size(); pid++) {
            const PatchInfo &p = c->patches[pid];
            if (st[p.scen].dt > 0.0) continue;
            long long n = (long long)p.nx * p.ny;
            const uint8_t *m = st[p.scen].cur ? c->m1 : c->m0;
            unsigned nb = (unsigned)((n + 255) / 256);
            if (c->mixed)
                initdt_kernel<float, true><<<nb, 256, 0, c->stream>>>(
                    p, c->P, st[p.scen].cur ? c->f1 : c->f0, c->fbath, m, c->d_slots + p.scen,
                    c->d_err);
            else
                initdt_kernel<double, false><<<nb, 256, 0, c->stream>>>(
                    p, c->P, st[p.scen].cur ? c->q1 : c->q0, c->bath, m, c->d_slots + p.scen,
                    c->d_err);
        }
        initdt_finish<<<(unsigned)((ns + 63) / 64), 64, 0, c->stream>>>(c->d_scen, c->d_sstat,
                                                                        c->d_slots, ns);
        HIPCHK(c, hipGetLastError());
        int err = 0;
        HIPCHK(c, hipMemcpyAsync(&err, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (err) return fail(c, err, "initial step: state not hyperbolic");
    }
    if ((rc = ensure_gauges(c, st, (long long)n_steps + 256))) return rc;
    long long attempts = n_steps, budget = (long long)n_steps + 4096;
    while (attempts > 0) {
        for (long long a = 0; a < attempts; a++) {
            if ((rc = launch_attempt(c))) return rc;
            if (c->timing && c->ev_used >= 8192 && (rc = collect_timing(c))) return rc;
        }
        budget -= attempts;
        if ((rc = pull_scen(c, st))) return rc;
        long long left = 0;
        for (size_t s = 0; s < st.size(); s++)
            if (st[s].active && !st[s].err) left = std::max(left, st[s].target - st[s].steps);
        if (left > 0 && budget > 0) {
            if ((rc = ensure_gauges(c, st, left + 256))) return rc;
            attempts = std::min(left, budget);
        } else {
            attempts = 0;
        }
    }
    for (size_t s = 0; s < st.size(); s++) {
        if (st[s].err) return fail(c, st[s].err, std::string("scenario ") + std::to_string(s) + ": " + hsgn_strerror(st[s].err));
        if (st[s].steps < st[s].target) return fail(c, HSGN_ECFL, "too many rejected steps");
    }
    return HSGN_OK;
}

int hsgn_diagnostics(hsgn_ctx *c, int scenario, hsgn_diag *d)
{
    if (!c || !c->finalized || !d) return fail(c, HSGN_EINVAL, "bad arguments");
    if (scenario < 0 || scenario >= (int)c->scen.size()) return fail(c, HSGN_EINVAL, "bad scenario");
    std::vector<ScenState> st;
    int rc = pull_scen(c, st);
    if (rc) return rc;
    memset(d, 0, sizeof(*d));
    const ScenState &s = st[scenario];
    double mass = 0.0;
    unsigned long long cnt_h[2] = {0, 0};
    long long cells = 0;
    unsigned long long *dcnt = nullptr;
    HIPCHK(c, hipMalloc(&dcnt, sizeof(unsigned long long) * 2));
    for (int pid : c->scen[scenario].patches) {
        const PatchInfo &p = c->patches[pid];
        const uint8_t *m = s.cur ? c->m1 : c->m0;
        if (c->mixed)
            mass_kernel<float, true><<<1, 1024, 0, c->stream>>>(p, s.cur ? c->f1 : c->f0,
                                                                 c->fbath, c->prm.eta0, c->d_mass);
        else
            mass_kernel<double, false><<<1, 1024, 0, c->stream>>>(p, s.cur ? c->q1 : c->q0,
                                                                  c->bath, c->prm.eta0, c->d_mass);
        double pm = 0.0;
        HIPCHK(c, hipMemcpyAsync(&pm, c->d_mass, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemsetAsync(dcnt, 0, sizeof(unsigned long long) * 2, c->stream));
        long long n = (long long)p.nx * p.ny;
        count_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(p, m, dcnt);
        unsigned long long ch[2];
        HIPCHK(c, hipMemcpyAsync(ch, dcnt, sizeof(ch), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        mass += pm * p.dx * p.dy;
        cnt_h[0] += ch[0];
        cnt_h[1] += ch[1];
        cells += n;
    }
    (void)hipFree(dcnt);
    d->mass = mass;
    d->clipped_mass = s.clip_total;
    d->max_courant = s.max_courant;
    d->last_courant = s.courant;
    d->steps = s.steps;
    d->rejected = s.rejects;
    d->cell_updates = s.steps * cells;
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
    st[scenario].t = t;
    st[scenario].dt = dt_next > 0.0 ? dt_next : 0.0;
    st[scenario].steps = steps;
    st[scenario].err = 0;
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
