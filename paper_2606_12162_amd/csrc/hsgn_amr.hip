// hsgn_amr.hip -- kernels of static patch sets: ghost fill, boundary-flux
// sums, refluxing and averaging down (rules in hsgn_amr.hpp).  Compiled
// without floating-point contraction, like the FP64 step kernel, so that the
// FP64 results round exactly as a plain evaluation of the same formulas.
#include "hsgn_amr.hpp"

namespace hsgn {

namespace {

constexpr int TPB = 128;

inline unsigned blocks(long long n) { return (unsigned)((n + TPB - 1) / TPB); }

__device__ inline bool scen_failed(const ScenState *S, int slot) { return S[slot].err != 0; }

// minmod of two slopes: the one of smaller magnitude if they agree in sign
__device__ inline double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a <= b ? a : b;
    if (a < 0.0 && b < 0.0) return a >= b ? a : b;
    return 0.0;
}

template <class S>
__global__ void halo_copy_kernel(AmrBuffers<S> B, const GhostCopy *R, int n)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const GhostCopy r = R[k];
    const PatchInfo D = B.patches[r.dp], Sp = B.patches[r.sp];
    if (scen_failed(B.scen, D.scen)) return;
    const int cur = B.scen[D.scen].cur;          // same level: same slot as the source
    S *q = cur ? B.q1 : B.q0;
    uint8_t *mk = cur ? B.m1 : B.m0;
    S v[7];
    for (int m = 0; m < 7; m++) v[m] = q[Sp.qoff + m * Sp.plane + r.sl];
    if (r.flips && Sp.metric) {
        // mapped: mirrored about the wall edge, the x wall first
        const long long MP = (long long)Sp.pitch * (Sp.ny + 4), base = 2LL * Sp.pitch + 2;
        double hu = (double)v[IHU], hv = (double)v[IHV];
        if (r.flips & 1) {
            const double *e = Sp.metric + base + r.wx;
            reflect(hu, hv, e[MP], e[2 * MP]);
        }
        if (r.flips & 2) {
            const double *e = Sp.metric + base + r.wy;
            reflect(hu, hv, e[4 * MP], e[5 * MP]);
        }
        v[IHU] = (S)hu;
        v[IHV] = (S)hv;
    } else {
        if (r.flips & 1) v[IHU] = -v[IHU];
        if (r.flips & 2) v[IHV] = -v[IHV];
    }
    for (int m = 0; m < 7; m++) q[D.qoff + m * D.plane + r.dl] = v[m];
    mk[D.coff + r.dl] = (uint8_t)(mk[Sp.coff + r.sl] & 3);
}

// eta', hu, ..., h p_b of a coarse cell at the old and new time levels, in
// FP64, and whether it is dry at either
template <class S, bool MIXED>
__device__ void coarse_cell(const AmrBuffers<S> &B, const PatchInfo &C, int cl, const S *qo,
                            const S *qn, double eta0, double dry_tol, double vo[7], double vn[7],
                            bool &dry)
{
    const double b = (double)B.bath[C.coff + cl];
    for (int m = 0; m < 7; m++) {
        vo[m] = (double)qo[C.qoff + m * C.plane + cl];
        vn[m] = (double)qn[C.qoff + m * C.plane + cl];
    }
    double ho, hn;
    if (MIXED) {
        ho = (vo[0] + eta0) - b;
        hn = (vn[0] + eta0) - b;
    } else {
        ho = vo[0];
        hn = vn[0];
        vo[0] = (vo[0] + b) - eta0;
        vn[0] = (vn[0] + b) - eta0;
    }
    dry = !(ho > dry_tol) || !(hn > dry_tol);
}

template <class S, bool MIXED>
__global__ void halo_interp_kernel(AmrBuffers<S> B, const GhostInterp *R, int n, double theta,
                                   double eta0, double dry_tol)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const GhostInterp r = R[k];
    const PatchInfo D = B.patches[r.dp];
    if (scen_failed(B.scen, D.scen)) return;
    const PatchInfo C = B.patches[r.cp[0]];
    const int ccur = B.scen[C.scen].cur;         // the coarse step is done: cur = new
    const S *qn = ccur ? B.q1 : B.q0;
    const S *qo = ccur ? B.q0 : B.q1;
    double v[5][7];
    bool have[5], any_dry = false;
    for (int s = 0; s < 5; s++) {
        have[s] = r.cp[s] >= 0;
        if (!have[s]) continue;
        const PatchInfo Cs = B.patches[r.cp[s]];
        double vo[7], vn[7];
        bool dry;
        coarse_cell<S, MIXED>(B, Cs, r.cl[s], qo, qn, eta0, dry_tol, vo, vn, dry);
        any_dry = any_dry || dry;
        for (int m = 0; m < 7; m++) v[s][m] = (1.0 - theta) * vo[m] + theta * vn[m];
    }
    const double ox = (double)r.ox, oy = (double)r.oy;
    double out[7];
    for (int m = 0; m < 7; m++) {
        double sx = 0.0, sy = 0.0;
        if (!any_dry) {
            if (have[1] && have[2]) sx = minmod(v[2][m] - v[0][m], v[0][m] - v[1][m]);
            if (have[3] && have[4]) sy = minmod(v[4][m] - v[0][m], v[0][m] - v[3][m]);
        }
        out[m] = (v[0][m] + ox * sx) + oy * sy;
    }
    const double bg = (double)B.bath[D.coff + r.dl];
    double h = (out[0] + eta0) - bg;
    if (MIXED) {
        if (!(h > 0.0)) out[0] = bg - eta0;      // depth clipped at zero
    } else {
        out[0] = h > 0.0 ? h : 0.0;
    }
    const int cur = B.scen[D.scen].cur;
    S *q = cur ? B.q1 : B.q0;
    for (int m = 0; m < 7; m++) q[D.qoff + m * D.plane + r.dl] = (S)out[m];
    const uint8_t *mc = ccur ? B.m1 : B.m0;
    uint8_t *md = cur ? B.m1 : B.m0;
    md[D.coff + r.dl] = (uint8_t)(mc[C.coff + r.cl[0]] & 3);
}

template <class S>
__global__ void ghost_bath_kernel(AmrBuffers<S> B, const GhostCopy *Cp, int nc,
                                  const GhostInterp *In, int ni)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < nc) {
        const GhostCopy r = Cp[k];
        const PatchInfo D = B.patches[r.dp], Sp = B.patches[r.sp];
        B.bath[D.coff + r.dl] = B.bath[Sp.coff + r.sl];
    } else if (k < nc + ni) {
        const GhostInterp r = In[k - nc];
        const PatchInfo D = B.patches[r.dp], C = B.patches[r.cp[0]];
        B.bath[D.coff + r.dl] = B.bath[C.coff + r.cl[0]];
    }
}

// mean of the 4 x 4 fine cells (rows outer, columns inner); on a mapped
// patch set sum(kap v) / sum(kap) in the same order.  bath_only with keep
// (mixed storage, flag per coarse patch whose state is set): the covered
// cell's stored eta' follows the new bottom so that its depth is kept, as
// the FP64 storage of h keeps it
template <bool MAPPED, class S>
__device__ inline double fine_mean(const S *v, const PatchInfo &F, long long l,
                                   const double (&kap)[AMR_RATIO * AMR_RATIO], double wsum)
{
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < AMR_RATIO; a++)
#pragma unroll
        for (int c = 0; c < AMR_RATIO; c++) {
            const double x = (double)v[l + (long long)a * F.pitch + c];
            if (MAPPED) s += kap[a * AMR_RATIO + c] * x;
            else s += x;
        }
    return MAPPED ? s / wsum : s * 0.0625;
}

template <bool MAPPED, class S>
__device__ void avgdown_one(AmrBuffers<S> &B, const AvgRec &r, const PatchInfo &F,
                            const PatchInfo &C, int bath_only, const uint8_t *keep)
{
    // capacities of the 4 x 4 fine cells (mapped), read once
    double kap[AMR_RATIO * AMR_RATIO], wsum = 0.0;
#pragma unroll
    for (int a = 0; a < AMR_RATIO; a++)
#pragma unroll
        for (int c = 0; c < AMR_RATIO; c++) {
            kap[a * AMR_RATIO + c] =
                MAPPED ? F.metric[2LL * F.pitch + 2 + r.fl + (long long)a * F.pitch + c] : 1.0;
            wsum += kap[a * AMR_RATIO + c];
        }
    if (bath_only) {
        const S bn = (S)fine_mean<MAPPED>(B.bath + F.coff, F, r.fl, kap, wsum);
        if (keep && keep[r.cp]) {
            S *qc = B.scen[C.scen].cur ? B.q1 : B.q0;
            const long long l = C.qoff + r.cl;
            qc[l] = (S)((double)qc[l] + ((double)bn - (double)B.bath[C.coff + r.cl]));
        }
        B.bath[C.coff + r.cl] = bn;
        return;
    }
    if (scen_failed(B.scen, C.scen) || scen_failed(B.scen, F.scen)) return;
    const S *qf = B.scen[F.scen].cur ? B.q1 : B.q0;
    S *qc = B.scen[C.scen].cur ? B.q1 : B.q0;
    for (int m = 0; m < 7; m++)
        qc[C.qoff + m * C.plane + r.cl] =
            (S)fine_mean<MAPPED>(qf + F.qoff + m * F.plane, F, r.fl, kap, wsum);
}

template <class S>
__global__ void avgdown_kernel(AmrBuffers<S> B, const AvgRec *R, int n, int bath_only,
                               const uint8_t *keep)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const AvgRec r = R[k];
    const PatchInfo F = B.patches[r.fp], C = B.patches[r.cp];
    if (F.metric) avgdown_one<true>(B, r, F, C, bath_only, keep);
    else avgdown_one<false>(B, r, F, C, bath_only, keep);
}

// one cell of the old state of a patch (the buffer the last step read), after
// its first source half step
template <class S, bool MIXED>
__device__ void old_cell(const AmrBuffers<S> &B, const StepParams &P, const PatchInfo &pi, int l,
                         Cell<double> &c)
{
    const ScenState &st = B.scen[pi.scen];
    const S *q = st.cur ? B.q0 : B.q1;            // after the swap: the other buffer
    const uint8_t *mk = st.cur ? B.m0 : B.m1;
    RawCell<double> raw;
    for (int m = 0; m < 7; m++) raw.q[m] = (double)q[pi.qoff + m * pi.plane + l];
    raw.b = (double)B.bath[pi.coff + l];
    raw.mk = mk[pi.coff + l];
    int phi, brk;
    prepare_cell<double, MIXED>(P, raw, 0.5 * st.dt, c, phi, brk);
}

template <int DIR, class S, bool MIXED>
__device__ void edge_dflux(const AmrBuffers<S> &B, const StepParams &P, const FluxRec &r,
                           double D[7])
{
    const PatchInfo F = B.patches[r.fp], C = B.patches[r.cp];
    Cell<double> cc, cg;
    old_cell<S, MIXED>(B, P, C, r.cl, cc);
    old_cell<S, MIXED>(B, P, F, r.gl, cg);
    Side<double> sc, sg;
    Waves<double> W;
    Eig<double> E;
    double am[7], ap[7];
    if (F.metric) {
        // mapped: solved in the frame of the fine edge, the left (bottom)
        // edge of the cell right of (above) the ghost on a low side and of
        // the ghost itself on a high side; rotated back and scaled by the
        // edge's length ratio
        const long long MP = (long long)F.pitch * (F.ny + 4);
        const long long el = r.gl + (r.low ? (DIR == 0 ? 1 : F.pitch) : 0);
        const double *e = F.metric + 2LL * F.pitch + 2 + el;
        const double nx = DIR == 0 ? e[MP] : e[4 * MP], ny = DIR == 0 ? e[2 * MP] : e[5 * MP];
        const double gm = DIR == 0 ? e[3 * MP] : e[6 * MP];
        const double tx = DIR == 0 ? 0.0 - ny : ny, ty = DIR == 0 ? nx : 0.0 - nx;
        mapped_side(P, cc.q, cc.b, cc.c2, cc.eta, nx, ny, tx, ty, sc);
        mapped_side(P, cg.q, cg.b, cg.c2, cg.eta, nx, ny, tx, ty, sg);
        if (r.low) riemann<0>(P, sc, sg, W, E);
        else riemann<0>(P, sg, sc, W, E);
        set_frame(W, E, nx, ny, tx, ty, gm);
        fluctuations<0>(W, am, ap);
        to_global(W, am);
        to_global(W, ap);
    } else {
        side_of<DIR>(cc, sc);
        side_of<DIR>(cg, sg);
        if (r.low) riemann<DIR>(P, sc, sg, W, E);
        else riemann<DIR>(P, sg, sc, W, E);
        fluctuations<DIR>(W, am, ap);
    }
    for (int m = 0; m < 7; m++) D[m] = r.low ? am[m] + ap[m] : -(am[m] + ap[m]);
}

template <class S, bool MIXED>
__global__ void bflux_kernel(AmrBuffers<S> B, StepParams P, const FluxRec *R, int n,
                             const double *E, double *Rg)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const FluxRec r = R[k];
    const PatchInfo F = B.patches[r.fp];
    if (scen_failed(B.scen, F.scen)) return;
    double D[7];
    if (r.dir == 0) edge_dflux<0, S, MIXED>(B, P, r, D);
    else edge_dflux<1, S, MIXED>(B, P, r, D);
    const long long e = (F.eoff + r.entry) * 7;
    for (int m = 0; m < 7; m++) Rg[e + m] = Rg[e + m] + (E[e + m] + D[m]);
}

template <class S, bool MIXED>
__global__ void reflux_kernel(AmrBuffers<S> B, StepParams P, const RefluxRec *R, int n,
                              const double *Rg, double *rclip)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const RefluxRec r = R[k];
    const PatchInfo C = B.patches[r.cp];
    if (scen_failed(B.scen, C.scen)) return;
    const ScenState &st = B.scen[C.scen];
    S *q = st.cur ? B.q1 : B.q0;
    const uint8_t mk = (st.cur ? B.m1 : B.m0)[C.coff + r.cl];
    const double b = (double)B.bath[C.coff + r.cl];
    double v[7];
    for (int m = 0; m < 7; m++) v[m] = (double)q[C.qoff + m * C.plane + r.cl];
    if (MIXED) v[0] = (v[0] + P.eta0) - b;
    const double dtdx = st.dt / C.dx, dtdy = st.dt / C.dy;
    // mapped: the records are fluxes times length ratios, divided here by the
    // cell's capacity
    const double kap = C.metric ? C.metric[2LL * C.pitch + 2 + r.cl] : 1.0;
    for (int e = 0; e < 4; e++) {
        if (r.fp[e] < 0) continue;
        const PatchInfo F = B.patches[r.fp[e]];
        const double *Rf = Rg + (F.eoff + r.e0[e]) * 7;
        double dtd = e < 2 ? dtdx : dtdy;
        if (C.metric) dtd = dtd / kap;
        for (int m = 0; m < 7; m++) {
            double s = ((Rf[m] + Rf[7 + m]) + Rf[14 + m]) + Rf[21 + m];
            double corr = dtd * (s * 0.0625);
            // fine patch to the left / below: the cell lies above the edge
            v[m] = (e == 0 || e == 2) ? v[m] + corr : v[m] - corr;
        }
    }
    double clip = 0.0;
    if (v[0] < 0.0) {
        clip = C.metric ? -v[0] * kap * C.dx * C.dy : -v[0] * C.dx * C.dy;
        v[0] = 0.0;
    }
    if (v[0] <= P.dry_tol)
        for (int m = 1; m < 7; m++) v[m] = 0.0;
    const int phi = mk & 1, brk = (mk >> 1) & 1;
    if (!phi || brk || v[0] <= P.dry_tol) {
        v[IHW] = 0.0; v[IHS] = 0.0; v[IHP] = 0.0; v[IHPB] = 0.0;
    }
    rclip[k] += clip;
    if (MIXED) v[0] = (v[0] + b) - P.eta0;
    for (int m = 0; m < 7; m++) q[C.qoff + m * C.plane + r.cl] = (S)v[m];
}

__global__ void iface_kernel(const PatchInfo *patches, const RefluxRec *R, int n, uint8_t *m0,
                             uint8_t *m1)
{
    int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const RefluxRec r = R[k];
    const PatchInfo C = patches[r.cp];
    int bits = 0;
    for (int e = 0; e < 4; e++)
        if (r.fp[e] >= 0) bits |= 1 << e;
    long long i = C.coff + r.cl;
    m0[i] = (uint8_t)((m0[i] & 3) | (bits << 2));
    m1[i] = (uint8_t)((m1[i] & 3) | (bits << 2));
}

__global__ void fill_zero_kernel(double *p, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---- regridding ----------------------------------------------------------

// flag of one interior cell of a level-l patch: a wet face neighbour inside
// the patch whose surface eta' = (h + b) - eta0 differs by more than tol
template <class S, bool MIXED>
__device__ inline bool surface_of(const PatchInfo &P, const S *q, const S *bath, int x, int y,
                                  double eta0, double dry_tol, double &e)
{
    const long long l = (long long)y * P.pitch + x;
    const double v = (double)q[P.qoff + l];
    const double b = (double)bath[P.coff + l];
    if (MIXED) {
        e = v;
        return ((v + eta0) - b) > dry_tol;
    }
    e = (v + b) - eta0;
    return v > dry_tol;
}

// the record holding launch cell k (records sorted by c0, the first at 0)
template <class R>
__device__ inline int record_of(const R *rec, int nr, long long k)
{
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rec[mid].c0 <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// the flags of every level-l patch (the rule of surface_of), one thread per flag
template <class S, bool MIXED>
__global__ void regrid_flag_kernel(const FlagRec *R, int nr, long long total, const S *q,
                                   const S *bath, uint8_t *out, double eta0, double dry_tol,
                                   double tol)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const FlagRec &r = R[record_of(R, nr, k)];
    const PatchInfo &P = r.p;
    const long long e = k - r.c0;
    const int x = (int)(e % P.nx), y = (int)(e / P.nx);
    double e0, e1;
    uint8_t f = 0;
    if (surface_of<S, MIXED>(P, q, bath, x, y, eta0, dry_tol, e0)) {
        const int nbx[4] = {x - 1, x + 1, x, x};
        const int nby[4] = {y, y, y - 1, y + 1};
        for (int s = 0; s < 4; s++) {
            if (nbx[s] < 0 || nbx[s] >= P.nx || nby[s] < 0 || nby[s] >= P.ny) continue;
            if (surface_of<S, MIXED>(P, q, bath, nbx[s], nby[s], eta0, dry_tol, e1) &&
                fabs(e1 - e0) > tol)
                f = 1;
        }
    }
    out[k] = f;
}

// copy one cell from the old storage; a wet cell whose bathymetry changed
// keeps its surface (depth clipped at zero), a dry cell keeps its depth; the
// breaking latch comes along, phi_T and the interface bits stay the new ones
template <class S, bool MIXED>
__global__ void regrid_copy_kernel(const RegridCopy<S> *R, int nr, long long total, S *q,
                                   const S *bath, uint8_t *m0, uint8_t *m1, double eta0,
                                   double dry_tol)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const RegridCopy<S> r = R[record_of(R, nr, k)];
    const long long e = k - r.c0;
    const int x = (int)(e % r.nx), y = (int)(e / r.nx);
    const long long sl = (long long)(r.sj0 + y) * r.src.pitch + (r.si0 + x);
    const long long dl = (long long)(r.dj0 + y) * r.dst.pitch + (r.di0 + x);
    for (int m = 1; m < 7; m++)
        q[r.dst.qoff + m * r.dst.plane + dl] = r.sq[r.src.qoff + m * r.src.plane + sl];
    S v0 = r.sq[r.src.qoff + sl];
    const double bo = (double)r.sb[r.src.coff + sl], bn = (double)bath[r.dst.coff + dl];
    if (bo != bn) {
        if (MIXED) {
            const double h = ((double)v0 + eta0) - bo;
            double h2 = h;
            if (h > dry_tol) {
                h2 = h + (bo - bn);
                if (!(h2 > 0.0)) h2 = 0.0;
            }
            v0 = (S)((h2 + bn) - eta0);
        } else if ((double)v0 > dry_tol) {
            const double h2 = (double)v0 + (bo - bn);
            v0 = (S)(h2 > 0.0 ? h2 : 0.0);
        }
    }
    q[r.dst.qoff + dl] = v0;
    const uint8_t lat = (uint8_t)(r.sm[r.src.coff + sl] & MASK_BRK);
    m0[r.dst.coff + dl] = (uint8_t)((m0[r.dst.coff + dl] & ~MASK_BRK) | lat);
    m1[r.dst.coff + dl] = (uint8_t)((m1[r.dst.coff + dl] & ~MASK_BRK) | lat);
}

// one cell of a new patch from its coarse parent: the ghost rule's spatial
// interpolation (minmod-limited slopes, zero if a stencil cell is dry) and the
// parent cell's breaking latch.  The stencil lies inside the parent (the new
// patch keeps one parent cell clear of the parent's edges).
template <class S, bool MIXED>
__global__ void regrid_interp_kernel(const RegridInterp *R, int nr, long long total, S *q,
                                     const S *bath, uint8_t *m0, uint8_t *m1, double eta0,
                                     double dry_tol)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const RegridInterp r = R[record_of(R, nr, k)];
    const long long e = k - r.c0;
    const int i = (int)(e % r.fine.nx), j = (int)(e / r.fine.nx);
    const int ic = r.ci0 + (i >> 2), jc = r.cj0 + (j >> 2);
    const PatchInfo C = r.coarse, F = r.fine;
    const int sx_[5] = {ic, ic - 1, ic + 1, ic, ic};
    const int sy_[5] = {jc, jc, jc, jc - 1, jc + 1};
    double v[5][7];
    bool any_dry = false;
    for (int s = 0; s < 5; s++) {
        const long long cl = (long long)sy_[s] * C.pitch + sx_[s];
        for (int m = 0; m < 7; m++) v[s][m] = (double)q[C.qoff + m * C.plane + cl];
        const double b = (double)bath[C.coff + cl];
        double h;
        if (MIXED) {
            h = (v[s][0] + eta0) - b;
        } else {
            h = v[s][0];
            v[s][0] = (h + b) - eta0;
        }
        any_dry = any_dry || !(h > dry_tol);
    }
    const double ox = ((double)(i & 3) + 0.5) / 4.0 - 0.5;
    const double oy = ((double)(j & 3) + 0.5) / 4.0 - 0.5;
    double out[7];
    for (int m = 0; m < 7; m++) {
        double sx = 0.0, sy = 0.0;
        if (!any_dry) {
            sx = minmod(v[2][m] - v[0][m], v[0][m] - v[1][m]);
            sy = minmod(v[4][m] - v[0][m], v[0][m] - v[3][m]);
        }
        out[m] = (v[0][m] + ox * sx) + oy * sy;
    }
    const long long fl = (long long)j * F.pitch + i;
    const double bf = (double)bath[F.coff + fl];
    const double h = (out[0] + eta0) - bf;
    if (MIXED) {
        if (!(h > 0.0)) out[0] = bf - eta0;
    } else {
        out[0] = h > 0.0 ? h : 0.0;
    }
    for (int m = 0; m < 7; m++) q[F.qoff + m * F.plane + fl] = (S)out[m];
    const uint8_t lat = (uint8_t)(m0[C.coff + (long long)jc * C.pitch + ic] & MASK_BRK);
    m0[F.coff + fl] = (uint8_t)((m0[F.coff + fl] & ~MASK_BRK) | lat);
    m1[F.coff + fl] = (uint8_t)((m1[F.coff + fl] & ~MASK_BRK) | lat);
}

// bilinear interpolant of the level-0 bathymetry at one cell centre, in
// level-0 index coordinates (exact in binary), clamped at the outer centres
template <class S>
__global__ void topo_kernel(const TopoRec *R, int nr, long long total, const double *B0, int NX,
                            int NY, S *bath)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const TopoRec r = R[record_of(R, nr, k)];
    const long long e = k - r.c0;
    const int i = (int)(e % r.p.nx), j = (int)(e / r.p.nx);
    const double sc = (double)(1LL << (2 * r.level));
    const double fy = ((double)(r.J0 + j) + 0.5) / sc - 0.5;
    int jj = (int)floor(fy);
    jj = jj < 0 ? 0 : (jj > NY - 2 ? NY - 2 : jj);
    double s = fy - jj;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    const double fx = ((double)(r.I0 + i) + 0.5) / sc - 0.5;
    int ii = (int)floor(fx);
    ii = ii < 0 ? 0 : (ii > NX - 2 ? NX - 2 : ii);
    double t = fx - ii;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double *r0 = B0 + (long long)jj * NX, *r1 = B0 + (long long)(jj + 1) * NX;
    const double b = (r0[ii] * (1.0 - t) + r0[ii + 1] * t) * (1.0 - s) +
                     (r1[ii] * (1.0 - t) + r1[ii + 1] * t) * s;
    bath[r.p.coff + (long long)j * r.p.pitch + i] = (S)b;
}

}  // namespace

void launch_halo_copy64(const AmrBuffers<double> &B, const GhostCopy *r, int n, hipStream_t s)
{
    if (n > 0) halo_copy_kernel<double><<<blocks(n), TPB, 0, s>>>(B, r, n);
}
void launch_halo_copy32(const AmrBuffers<float> &B, const GhostCopy *r, int n, hipStream_t s)
{
    if (n > 0) halo_copy_kernel<float><<<blocks(n), TPB, 0, s>>>(B, r, n);
}
void launch_halo_interp64(const AmrBuffers<double> &B, const GhostInterp *r, int n, double theta,
                          double eta0, double dry_tol, hipStream_t s)
{
    if (n > 0)
        halo_interp_kernel<double, false><<<blocks(n), TPB, 0, s>>>(B, r, n, theta, eta0, dry_tol);
}
void launch_halo_interp32(const AmrBuffers<float> &B, const GhostInterp *r, int n, double theta,
                          double eta0, double dry_tol, hipStream_t s)
{
    if (n > 0)
        halo_interp_kernel<float, true><<<blocks(n), TPB, 0, s>>>(B, r, n, theta, eta0, dry_tol);
}
void launch_ghost_bath64(const AmrBuffers<double> &B, const GhostCopy *c, int nc,
                         const GhostInterp *r, int ni, hipStream_t s)
{
    if (nc + ni > 0) ghost_bath_kernel<double><<<blocks(nc + ni), TPB, 0, s>>>(B, c, nc, r, ni);
}
void launch_ghost_bath32(const AmrBuffers<float> &B, const GhostCopy *c, int nc,
                         const GhostInterp *r, int ni, hipStream_t s)
{
    if (nc + ni > 0) ghost_bath_kernel<float><<<blocks(nc + ni), TPB, 0, s>>>(B, c, nc, r, ni);
}
void launch_avgdown64(const AmrBuffers<double> &B, const AvgRec *r, int n, bool bath_only,
                      hipStream_t s)
{
    if (n > 0) avgdown_kernel<double><<<blocks(n), TPB, 0, s>>>(B, r, n, bath_only ? 1 : 0, nullptr);
}
void launch_avgdown32(const AmrBuffers<float> &B, const AvgRec *r, int n, bool bath_only,
                      hipStream_t s, const uint8_t *keep)
{
    if (n > 0) avgdown_kernel<float><<<blocks(n), TPB, 0, s>>>(B, r, n, bath_only ? 1 : 0, keep);
}
void launch_bflux64(const AmrBuffers<double> &B, const StepParams &P, const FluxRec *r, int n,
                    const double *E, double *R, hipStream_t s)
{
    if (n > 0) bflux_kernel<double, false><<<blocks(n), TPB, 0, s>>>(B, P, r, n, E, R);
}
void launch_bflux32(const AmrBuffers<float> &B, const StepParams &P, const FluxRec *r, int n,
                    const double *E, double *R, hipStream_t s)
{
    if (n > 0) bflux_kernel<float, true><<<blocks(n), TPB, 0, s>>>(B, P, r, n, E, R);
}
void launch_reflux64(const AmrBuffers<double> &B, const StepParams &P, const RefluxRec *r, int n,
                     const double *R, double *rclip, hipStream_t s)
{
    if (n > 0) reflux_kernel<double, false><<<blocks(n), TPB, 0, s>>>(B, P, r, n, R, rclip);
}
void launch_reflux32(const AmrBuffers<float> &B, const StepParams &P, const RefluxRec *r, int n,
                     const double *R, double *rclip, hipStream_t s)
{
    if (n > 0) reflux_kernel<float, true><<<blocks(n), TPB, 0, s>>>(B, P, r, n, R, rclip);
}
void launch_iface(const PatchInfo *patches, const RefluxRec *r, int n, uint8_t *m0, uint8_t *m1,
                  hipStream_t s)
{
    if (n > 0) iface_kernel<<<blocks(n), TPB, 0, s>>>(patches, r, n, m0, m1);
}
void launch_fill_zero(double *p, long long n, hipStream_t s)
{
    if (n > 0) fill_zero_kernel<<<blocks(n), TPB, 0, s>>>(p, n);
}

void launch_regrid_flag64(const FlagRec *r, int nr, long long total, const double *q,
                          const double *bath, uint8_t *out, double eta0, double dry_tol,
                          double tol, hipStream_t s)
{
    if (nr > 0 && total > 0)
        regrid_flag_kernel<double, false><<<blocks(total), TPB, 0, s>>>(r, nr, total, q, bath, out,
                                                                        eta0, dry_tol, tol);
}
void launch_regrid_flag32(const FlagRec *r, int nr, long long total, const float *q,
                          const float *bath, uint8_t *out, double eta0, double dry_tol,
                          double tol, hipStream_t s)
{
    if (nr > 0 && total > 0)
        regrid_flag_kernel<float, true><<<blocks(total), TPB, 0, s>>>(r, nr, total, q, bath, out,
                                                                      eta0, dry_tol, tol);
}
void launch_regrid_copy64(const RegridCopy<double> *r, int nr, long long total, double *q,
                          const double *bath, uint8_t *m0, uint8_t *m1, double eta0,
                          double dry_tol, hipStream_t s)
{
    if (nr > 0 && total > 0)
        regrid_copy_kernel<double, false><<<blocks(total), TPB, 0, s>>>(r, nr, total, q, bath, m0,
                                                                        m1, eta0, dry_tol);
}
void launch_regrid_copy32(const RegridCopy<float> *r, int nr, long long total, float *q,
                          const float *bath, uint8_t *m0, uint8_t *m1, double eta0,
                          double dry_tol, hipStream_t s)
{
    if (nr > 0 && total > 0)
        regrid_copy_kernel<float, true><<<blocks(total), TPB, 0, s>>>(r, nr, total, q, bath, m0,
                                                                      m1, eta0, dry_tol);
}
void launch_regrid_interp64(const RegridInterp *r, int nr, long long total, double *q,
                            const double *bath, uint8_t *m0, uint8_t *m1, double eta0,
                            double dry_tol, hipStream_t s)
{
    if (nr > 0 && total > 0)
        regrid_interp_kernel<double, false><<<blocks(total), TPB, 0, s>>>(r, nr, total, q, bath, m0,
                                                                          m1, eta0, dry_tol);
}
void launch_regrid_interp32(const RegridInterp *r, int nr, long long total, float *q,
                            const float *bath, uint8_t *m0, uint8_t *m1, double eta0,
                            double dry_tol, hipStream_t s)
{
    if (nr > 0 && total > 0)
        regrid_interp_kernel<float, true><<<blocks(total), TPB, 0, s>>>(r, nr, total, q, bath, m0,
                                                                        m1, eta0, dry_tol);
}

void launch_topo64(const TopoRec *r, int nr, long long total, const double *B0, int NX, int NY,
                   double *bath, hipStream_t s)
{
    if (nr > 0 && total > 0)
        topo_kernel<double><<<blocks(total), TPB, 0, s>>>(r, nr, total, B0, NX, NY, bath);
}
void launch_topo32(const TopoRec *r, int nr, long long total, const double *B0, int NX, int NY,
                   float *bath, hipStream_t s)
{
    if (nr > 0 && total > 0)
        topo_kernel<float><<<blocks(total), TPB, 0, s>>>(r, nr, total, B0, NX, NY, bath);
}

}  // namespace hsgn
