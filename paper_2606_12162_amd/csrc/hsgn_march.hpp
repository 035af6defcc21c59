// hsgn_march.hpp -- one wavefront advances one strip of a patch by one step.
//
// Mapping: lane l of a 64-wide wavefront owns column i0 - 2 + l of a patch,
// so a wavefront covers 60 interior columns plus two halo columns on each
// side.  It marches up the rows r0 - 2 .. r0 + th + 1 of its strip, loading
// one row per iteration (coalesced SoA loads), and writes rows r0 .. r0+th-1.
// x-neighbours are exchanged with lane shuffles; y-neighbours live in
// registers (sliding windows).  Each wavefront keeps its own LDS area (the
// x-edge eigenstructure of three rows, in mixed precision the rows' base
// states, in FP64 the values parked between rows); a lane touches only its
// own entries, so no barrier is needed and a wavefront is independent of
// every other.
//
// Per iteration k (row k loaded):
//   1. load cell (i, k) through the boundary map, first source half step;
//   2. x-edge (i-1/2, k): normal solve, limiter (neighbour waves by
//      shuffle), net fluctuation entering cell (i, k);
//   3. y-edge (i, k-1/2): normal solve; finish the limiter of the y-edge
//      below it and feed its fluctuations to rows k-1 and k-2;
//   4. transverse terms: the x-fluctuations entering cells (i, k-1) and
//      (i, k) split by the y-edge (i, k-1/2); the y-fluctuations entering
//      cells (i-1, k-2) and (i, k-2) split by the x-edge (i-1/2, k-2);
//   5. row k-2 is complete: second source half step, fix-ups, store.
//
// The transverse terms of a cell are split once for the sum of the
// fluctuations entering it from its two edges in the other direction; by
// linearity of the split this equals splitting each edge's fluctuation.
#pragma once

#include "hsgn_math.hpp"

namespace hsgn {

struct PatchInfo {
    int nx, ny, pitch, scen;
    int bc[4];               // x-low, x-high, y-low, y-high
    double dx, dy;
    long long qoff;          // element offset of interior cell (0, 0) in plane 0
    long long coff;          // element offset of interior cell (0, 0) in the
                             // bathymetry / mask plane
    long long plane;         // elements per state plane
    long long eoff;          // offset (in 7-vectors) of the patch's boundary-flux
                             // entries, -1 if it has none
    int level, frame;        // refinement level; 2 if ghost cells are stored
    // sponge layer: widths (m) from the domain's x-low, x-high, y-low, y-high
    // sides (0: none), peak rate (1/s; 0: no sponge), and the patch's place
    // in the domain of its level (global index of interior cell (0, 0),
    // domain size in cells)
    double sp_w[4], sp_rate;
    long long sp_i0, sp_j0, sp_nx, sp_ny;
    // mapped grid (Sec. 4, mapped grids; single grids and patch sets), else null:
    // 7 planes of (ny + 4) x (nx + 4) values over the cells with their two
    // ghost layers, cell (i, j) at (j + 2) (nx + 4) + i + 2: capacity; unit
    // normal (x, y) and length ratio of the cell's left edge; the same for
    // its bottom edge
    const double *metric;
};

// relaxation rate of the sponge at interior cell (i, j) of a patch: with d
// the distance of the cell centre from a sponged side and w that side's
// width, s = (w - d) / w inside the band; the largest s over the sides gives
// rate s^2
HSGN_HD double sponge_sigma(const PatchInfo &pi, int i, int j)
{
    const long long I = pi.sp_i0 + i, J = pi.sp_j0 + j;
    const double d[4] = {((double)I + 0.5) * pi.dx, ((double)(pi.sp_nx - 1 - I) + 0.5) * pi.dx,
                         ((double)J + 0.5) * pi.dy, ((double)(pi.sp_ny - 1 - J) + 0.5) * pi.dy};
    double s = 0.0;
    for (int e = 0; e < 4; e++) {
        const double w = pi.sp_w[e];
        if (w > 0.0 && d[e] < w) {
            const double t = (w - d[e]) / w;
            if (t > s) s = t;
        }
    }
    return pi.sp_rate * (s * s);
}

// mask byte bits: phi_T, breaking latch, and the four edges of a cell whose
// contributions a finer patch replaces (patch sets)
constexpr int MASK_PHI = 1, MASK_BRK = 2;
constexpr int IFACE_L = 1, IFACE_R = 2, IFACE_B = 4, IFACE_T = 8;   // (mask >> 2)

struct WorkItem {
    int patch, i0, r0, th;   // strip: columns i0..i0+59, rows r0..r0+th-1; a packed
                             // item: patch = -1 - its PackedItem, th its tallest tile
};

// Narrow strips of patch-set patches packed into one wavefront: strip s
// (s < nseg) covers columns i0[s] .. i0[s] + w - 1 of patch[s] (w = min(60,
// nx - i0[s]) < 60) and rows r0[s] .. r0[s] + th[s] - 1, on lanes l0[s] ..
// l0[s] + w + 3 (two halo columns on either side).  All strips of an item
// lie in patches of one refinement level of one scenario (one clock slot).
constexpr int PACK_SEGS = 4;
struct PackedItem {
    int nseg;
    int patch[PACK_SEGS], i0[PACK_SEGS], r0[PACK_SEGS], th[PACK_SEGS], l0[PACK_SEGS];
};

// the strip a lane works on and its first lane
struct LaneStrip {
    int patch, i0, r0, th, l0;
};

// per-scenario clock and control, device resident
struct ScenState {
    double t, dt, dt_fixed, courant, max_courant;
    double rx, ry;           // max |speed| over x- and y-edges of the attempt
    long long steps, rejects, target, records;
    int cur;                 // which state buffer holds Q^n
    int active;              // step kernels work on this scenario
    int err;                 // sticky error code
    int accepted;            // the last attempt was accepted
    int adaptive;
    int streak;              // consecutive rejected attempts
    unsigned long long rx_bits, ry_bits;
    double clip_total;
};

// S: storage type of the state and bathymetry planes.  With FP64 storage
// plane 0 holds h; with FP32 storage it holds the surface deviation
// eta' = h + b - eta0.
template <class S>
struct MarchArgs {
    StepParams P;
    const PatchInfo *patches;
    const WorkItem *work;
    const PackedItem *packs; // strips of the packed items (patch sets), or null
    S *q0, *q1;              // state buffers (ping-pong)
    const S *bath;
    uint8_t *m0, *m1;        // mask buffers (ping-pong): bit0 phi_T, bit1 breaking
    ScenState *scen;
    double *clip_slots;      // one per work item
    double *eflux;           // boundary-edge fluxes of patches with eoff >= 0
    // split step (mixed-precision single grids), else null: the items none
    // of whose edges takes the FP64 solve (no cell they load has c^2 = 0)
    // listed in list[0 .. lcnt[0]), the others in list[nwork .. nwork +
    // lcnt[1]); clsb per item 1 when the bottom alone gives a cell it loads
    // c^2 = 0 (static between bathymetry changes)
    int *list;
    unsigned *lcnt;
    const int *clsb;
    // split step over single grids only: set to 1 by a step kernel that
    // latches a cell as breaking (the only change of the classes within an
    // advance); with it 0 the classification keeps the previous lists.  Null:
    // every attempt classifies.
    int *latch;
    int sponge;              // some patch has a sponge: the kernels compiled with it
    int mapped;              // some patch is mapped: the kernel compiled for it
    int nwork;
};

// a plain item is one strip over the whole wavefront; in a packed item each
// lane takes the strip whose lanes hold it (lanes past the last strip's
// belong to it, as idle lanes of a partial strip)
template <class S>
HSGN_HD LaneStrip lane_strip(const MarchArgs<S> &A, const WorkItem &wk, int lane)
{
    LaneStrip ls = {wk.patch, wk.i0, wk.r0, wk.th, 0};
    if (wk.patch < 0) {
        const PackedItem &pk = A.packs[-1 - wk.patch];
        int s = 0;
        HSGN_UNROLL
        for (int t = 1; t < PACK_SEGS; t++) s += (t < pk.nseg && lane >= pk.l0[t]) ? 1 : 0;
        ls = {pk.patch[s], pk.i0[s], pk.r0[s], pk.th[s], pk.l0[s]};
    }
    return ls;
}

// a patch of the item's clock slot
template <class S>
HSGN_HD int item_patch(const MarchArgs<S> &A, const WorkItem &wk)
{
    return wk.patch >= 0 ? wk.patch : A.packs[-1 - wk.patch].patch[0];
}

template <class L, class T>
HSGN_HD void shfl_side_up(L &ln, const Side<T> &c, Side<T> &o)
{
    o.h = ln.up(c.h); o.sq = ln.up(c.sq); o.ce = ln.up(c.ce);
    o.hun = ln.up(c.hun); o.un = ln.up(c.un); o.ut = ln.up(c.ut);
    o.w = ln.up(c.w); o.s = ln.up(c.s); o.p = ln.up(c.p); o.pb = ln.up(c.pb);
    o.hp = ln.up(c.hp); o.b = ln.up(c.b); o.c2 = ln.up(c.c2); o.eta = ln.up(c.eta);
    o.wet = ln.upi(c.wet); o.hyp = ln.upi(c.hyp);
}

// x-edge eigenstructure kept for two rows in a per-wavefront LDS ring
// (3 row slots x EIG_FIELDS x 64 lanes); each lane only touches its own
// entries, so no synchronisation is needed
constexpr int EIG_FIELDS = 13;

template <bool MAP = false, class T>
HSGN_HD void eig_store(T *ring, int slot, int lane, const Eig<T> &e)
{
    T *p = ring + (slot * (EIG_FIELDS + (MAP ? 5 : 0))) * 64 + lane;
    if (MAP) {
        p[13 * 64] = e.fnx; p[14 * 64] = e.fny; p[15 * 64] = e.ftx; p[16 * 64] = e.fty;
        p[17 * 64] = e.gm;
    }
    p[0 * 64] = e.uh; p[1 * 64] = e.vh; p[2 * 64] = e.wh; p[3 * 64] = e.sh;
    p[4 * 64] = e.pbh; p[5 * 64] = e.ghh; p[6 * 64] = e.c2p; p[7 * 64] = e.inv_ce2;
    p[8 * 64] = e.smin; p[9 * 64] = e.smax; p[10 * 64] = e.inv_ds;
    p[11 * 64] = e.wet ? (T)1 : (T)0; p[12 * 64] = e.ce2;
}

template <bool MAP = false, class T>
HSGN_HD void eig_load(const T *ring, int slot, int lane, Eig<T> &e)
{
    const T *p = ring + (slot * (EIG_FIELDS + (MAP ? 5 : 0))) * 64 + lane;
    if (MAP) {
        e.fnx = p[13 * 64]; e.fny = p[14 * 64]; e.ftx = p[15 * 64]; e.fty = p[16 * 64];
        e.gm = p[17 * 64];
    }
    e.uh = p[0 * 64]; e.vh = p[1 * 64]; e.wh = p[2 * 64]; e.sh = p[3 * 64];
    e.pbh = p[4 * 64]; e.ghh = p[5 * 64]; e.c2p = p[6 * 64]; e.inv_ce2 = p[7 * 64];
    e.smin = p[8 * 64]; e.smax = p[9 * 64]; e.inv_ds = p[10 * 64];
    e.wet = p[11 * 64] != (T)0; e.ce2 = p[12 * 64];
}

// values parked in a per-wavefront LDS area between rows, two per lane and
// access: entry j of lane l at pair j * 64 + l
template <class T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};
constexpr int PARK_WAVES = 24, PARK_SIDE = 14;

template <class T>
HSGN_HD void park_waves(T *buf, int lane, const Waves<T> &w)
{
    const T v[PARK_WAVES] = {w.z0[0], w.z0[1], w.z0[2], w.z0[3], w.z0[4], w.z0[5], w.z0[6],
                             w.z6[0], w.z6[1], w.z6[2], w.z6[3], w.z6[4], w.z6[5], w.z6[6],
                             w.zm[0], w.zm[1], w.zm[2], w.bs, w.bw, w.bt, w.bpb,
                             w.smin, w.smax, w.uh};
    Pair<T> *p = reinterpret_cast<Pair<T> *>(buf);
    HSGN_UNROLL
    for (int j = 0; j < PARK_WAVES / 2; j++) p[j * 64 + lane] = Pair<T>{v[2 * j], v[2 * j + 1]};
}

template <class T>
HSGN_HD void unpark_waves(const T *buf, int lane, int kind, Waves<T> &w)
{
    T v[PARK_WAVES];
    const Pair<T> *p = reinterpret_cast<const Pair<T> *>(buf);
    HSGN_UNROLL
    for (int j = 0; j < PARK_WAVES / 2; j++) {
        const Pair<T> x = p[j * 64 + lane];
        v[2 * j] = x.a;
        v[2 * j + 1] = x.b;
    }
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) { w.z0[m] = v[m]; w.z6[m] = v[7 + m]; }
    w.zm[0] = v[14]; w.zm[1] = v[15]; w.zm[2] = v[16];
    w.bs = v[17]; w.bw = v[18]; w.bt = v[19]; w.bpb = v[20];
    w.smin = v[21]; w.smax = v[22]; w.uh = v[23];
    w.kind = kind;
}

template <class T>
HSGN_HD void park_side(T *buf, int lane, const Side<T> &d)
{
    const T v[PARK_SIDE] = {d.h, d.sq, d.ce, d.hun, d.un, d.ut, d.w,
                            d.s, d.p, d.pb, d.hp, d.b, d.c2, d.eta};
    Pair<T> *p = reinterpret_cast<Pair<T> *>(buf);
    HSGN_UNROLL
    for (int j = 0; j < PARK_SIDE / 2; j++) p[j * 64 + lane] = Pair<T>{v[2 * j], v[2 * j + 1]};
}

template <class T>
HSGN_HD void unpark_side(const T *buf, int lane, int wet, int hyp, Side<T> &d)
{
    T v[PARK_SIDE];
    const Pair<T> *p = reinterpret_cast<const Pair<T> *>(buf);
    HSGN_UNROLL
    for (int j = 0; j < PARK_SIDE / 2; j++) {
        const Pair<T> x = p[j * 64 + lane];
        v[2 * j] = x.a;
        v[2 * j + 1] = x.b;
    }
    d.h = v[0]; d.sq = v[1]; d.ce = v[2]; d.hun = v[3]; d.un = v[4]; d.ut = v[5]; d.w = v[6];
    d.s = v[7]; d.p = v[8]; d.pb = v[9]; d.hp = v[10]; d.b = v[11]; d.c2 = v[12]; d.eta = v[13];
    d.wet = wet;
    d.hyp = hyp;
}

template <bool MAP = false, class L, class T>
HSGN_HD void shfl_waves_up(L &ln, const Waves<T> &w, Waves<T> &o)
{
    if (MAP) {
        o.fnx = ln.up(w.fnx); o.fny = ln.up(w.fny); o.ftx = ln.up(w.ftx); o.fty = ln.up(w.fty);
        o.gm = ln.up(w.gm);
    }
    for (int m = 0; m < 7; m++) { o.z0[m] = ln.up(w.z0[m]); o.z6[m] = ln.up(w.z6[m]); }
    for (int m = 0; m < 3; m++) o.zm[m] = ln.up(w.zm[m]);
    o.bs = ln.up(w.bs); o.bw = ln.up(w.bw); o.bt = ln.up(w.bt); o.bpb = ln.up(w.bpb);
    o.smin = ln.up(w.smin); o.smax = ln.up(w.smax); o.uh = ln.up(w.uh);
    o.kind = ln.upi(w.kind);
}

template <class L, class T>
HSGN_HD void shfl_vec(L &ln, const T *a, T *o, bool up)
{
    for (int m = 0; m < 7; m++) o[m] = up ? ln.up(a[m]) : ln.dn(a[m]);
}

// raw data of one cell as stored (state plane 0 as stored, bathymetry,
// mask byte), converted to the compute type, and the wall mirror still to be
// applied to it (mirror_raw): flip the x- (fx of the column) or the y-momentum
// (fy), on mapped grids reflect about the wall edge of unit normal wn (x) or
// bn (y)
template <class T>
struct RawCell {
    T q[7];
    T b;
    int mk;
    int fy;
    T wn[2], bn[2];
};

// m - 2 (m . n) n: momentum (hu, hv) mirrored about a wall of unit normal n
template <class T>
HSGN_HD void reflect(T &hu, T &hv, T nx, T ny)
{
    const T a = hu * nx + hv * ny;
    hu = hu - (T)2 * a * nx;
    hv = hv - (T)2 * a * ny;
}

// load cell (col, row) of a patch through the boundary map, or (FRAMED)
// from the stored ghost frame.  On a mapped grid a wall mirrors the
// momentum about the wall edge of the interior cell's row (column): the
// left edge of column xwall (0 or nx), the bottom edge of row 0 or ny.  The
// mirror is applied by mirror_raw when the cell is used: applied here it
// would make the next row's prefetch wait for its own loads.
template <bool FRAMED, bool MAP = false, class S, class T>
HSGN_HD void load_raw(const PatchInfo &pi, const S *q, const S *bath, const uint8_t *mask,
                      int mc, int fx, int row, RawCell<T> &r, int xwall = 0)
{
    int fy = 0;
    int mr = FRAMED ? row : map_index(row, pi.ny, pi.bc[2], pi.bc[3], &fy);
    long long idx = (long long)mr * pi.pitch + mc;
    long long plane = pi.plane;
    const S *qp = q + pi.qoff + idx;
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) r.q[m] = (T)qp[m * plane];
    r.fy = fy;
    if (MAP && pi.metric) {
        const long long W = pi.nx + 4, MP = W * (pi.ny + 4);
        if (fx) {
            const double *e = pi.metric + (long long)(mr + 2) * W + (xwall + 2);
            r.wn[0] = (T)e[1 * MP];
            r.wn[1] = (T)e[2 * MP];
        }
        if (fy) {
            const double *e = pi.metric + (long long)((row < 0 ? 0 : pi.ny) + 2) * W + (mc + 2);
            r.bn[0] = (T)e[4 * MP];
            r.bn[1] = (T)e[5 * MP];
        }
    }
    r.b = (T)bath[pi.coff + idx];
    r.mk = mask[pi.coff + idx];
}

// the wall mirror recorded by load_raw (fx: the column's)
template <bool MAP, class T>
HSGN_HD void mirror_raw(RawCell<T> &r, int fx, bool mapped)
{
    if (MAP && mapped) {
        if (fx) reflect(r.q[IHU], r.q[IHV], r.wn[0], r.wn[1]);
        if (r.fy) reflect(r.q[IHU], r.q[IHV], r.bn[0], r.bn[1]);
    } else {
        if (fx) r.q[IHU] = -r.q[IHU];
        if (r.fy) r.q[IHV] = -r.q[IHV];
    }
}

// depth from the stored plane-0 value
template <class T, bool MIXED>
HSGN_HD T depth_of(const StepParams &P, T q0, T b)
{
    return MIXED ? q0 + (T)P.eta0 - b : q0;
}

// relaxation parameter c^2 of a cell from its mask byte and bottom: zero in
// the SWE region (phi_T = 0) and in a breaking cell
template <class T>
HSGN_HD T relax_c2(const StepParams &P, int mk, T b)
{
    int swe = !(mk & MASK_PHI) || (mk & MASK_BRK);
    return swe ? (T)0 : (T)P.a2g * still_depth(P, b) + (T)P.c2f;
}

// apply the first source half step (Strang) or clear a dry/SWE cell's
// auxiliaries, then derive the primitive variables
template <class T, bool MIXED>
HSGN_HD void prepare_cell(const StepParams &P, const RawCell<T> &r, T tau_pre, Cell<T> &c,
                          int &phi, int &brk)
{
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) c.q[m] = r.q[m];
    c.b = r.b;
    c.q[IH] = depth_of<T, MIXED>(P, r.q[IH], r.b);
    phi = r.mk & 1;
    brk = (r.mk >> 1) & 1;
    int swe = !phi || brk;
    c.c2 = relax_c2(P, r.mk, c.b);
    if (P.splitting) {
        source_or_clear(P, c.q, c.c2, swe, tau_pre);
    } else if (!(c.q[IH] > (T)P.dry_tol) || swe) {
        c.q[IHW] = (T)0; c.q[IHS] = (T)0; c.q[IHP] = (T)0; c.q[IHPB] = (T)0;
    }
    derive(P, c);
    c.eta = MIXED ? r.q[IH] : c.h + c.b;
}

// one side of a mapped edge: the cell's state (after the first source half
// step) with its momentum rotated into the edge's frame (unit normal n,
// tangent t), its primitives derived from the rotated state; eta is the
// cell's surface for the hydrostatic jump (unchanged by the rotation)
template <class T>
HSGN_HD void mapped_side(const StepParams &P, const T *q, T b, T c2, T eta, T nx, T ny, T tx,
                         T ty, Side<T> &sd)
{
    Cell<T> c;
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) c.q[m] = q[m];
    c.q[IHU] = q[IHU] * nx + q[IHV] * ny;
    c.q[IHV] = q[IHU] * tx + q[IHV] * ty;
    c.b = b;
    c.c2 = c2;
    derive(P, c);
    c.eta = eta;
    side_of<0>(c, sd);
}

// mapped edge: the frame and length ratio kept with the waves and the Roe
// state, the speeds scaled
template <class T>
HSGN_HD void set_frame(Waves<T> &W, Eig<T> &E, T nx, T ny, T tx, T ty, T gm)
{
    W.fnx = nx; W.fny = ny; W.ftx = tx; W.fty = ty; W.gm = gm;
    E.fnx = nx; E.fny = ny; E.ftx = tx; E.fty = ty; E.gm = gm;
    W.smin = W.smin * gm; W.smax = W.smax * gm; W.uh = W.uh * gm;
}

// a frame vector (a fluctuation) rotated to the global frame and scaled
template <class T>
HSGN_HD void to_global(const Waves<T> &W, T *v)
{
    const T hu = v[IHU] * W.fnx + v[IHV] * W.ftx;
    const T hv = v[IHU] * W.fny + v[IHV] * W.fty;
    v[IHU] = hu; v[IHV] = hv;
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) v[m] = v[m] * W.gm;
}

// normal solve of an edge.  In mixed precision an edge with an SWE or dry
// side (c^2 = 0 on a side) is solved again in FP64 from the promoted sides
// and its results replace the FP32 ones.
// FB false: the FP32 solve alone, for work items whose cells all have
// c^2 > 0 (the FP64 branch would never be taken).
// A wavefront none of whose used edges (use) has a dry side takes the solve
// compiled for two wet sides: the general one sets the dry-dry outputs
// before its branch, some 35 moves per edge on every row.
template <int DIR, bool MIXED, class L, class T>
HSGN_HD bool edge_solve(L &ln, const StepParams &P, const Side<T> &sl, const Side<T> &sr,
                        Waves<T> &W, Eig<T> &E, bool use = true)
{
    bool ok;
    if (ln.any(use && !(sl.wet && sr.wet))) ok = riemann<DIR>(P, sl, sr, W, E);
    else ok = riemann<DIR, true>(P, sl, sr, W, E);
    if (MIXED) {
        int need = !(sl.c2 > (T)0) || !(sr.c2 > (T)0);
        if (ln.any(need)) {
            Side<double> dl, dr;
            convert(sl, dl);
            convert(sr, dr);
            Waves<double> Wd;
            Eig<double> Ed;
            bool okd = riemann<DIR>(P, dl, dr, Wd, Ed);
            if (need) {
                convert(Wd, W);
                convert(Ed, E);
                ok = okd;
            }
        }
    }
    return ok;
}

// Lanes policy L provides: lane(), up(x)/dn(x) (value of lane-1 / lane+1)
// for float, double and int (upi/dni), any(pred) over the wavefront, ring()
// (the wavefront's LDS ring of 3 * EIG_FIELDS * 64 compute values, followed
// in mixed precision by 3 * 7 * 64 more for the rows' base states, and in
// FP64 on Cartesian grids by (PARK_WAVES + PARK_SIDE) * 64 for the values
// parked between rows), and
// finish(args, wave, scenario, rx, ry, clip) which reduces over the
// wavefront and publishes the results.
//
// AMR: patches of a patch set.  Their ghost cells are stored (filled before
// the step), a cell's update leaves out what reaches it through an edge
// flagged in its mask byte (a finer patch replaces it by refluxing), and the
// boundary edges of a patch with eoff >= 0 record what they send through
// the edge, relative to the flux function of the outside cell:
//   left  A-dQ + F~ + F~tr,   right -(A+dQ - F~) + F~tr,
//   below B-dQ + G~ + G~tr,   above -(B+dQ - G~) + G~tr
// at entries j, ny + j, 2 ny + i, 2 ny + nx + i of the patch.
// MAP: compiled for mapped grids: every edge is solved in its own frame; a
// patch without a metric takes the identity frames, unit ratios and
// capacities, which give the Cartesian results.  With AMR the boundary
// records hold the mapped contributions (global frame, scaled by the edge's
// length ratio).
template <class L, class S, class T, bool MIXED, bool AMR, bool FB = true, bool SP = false,
          bool MAP = false>
HSGN_HD void march(L &ln, const MarchArgs<S> &A, int wid)
{
    const WorkItem wk = A.work[wid];
    const int lane = ln.lane();
    // the lane's strip (patch sets: packed items hold several); the item's
    // clock slot, spacing and step are its first patch's.  Mapped patch sets
    // in mixed precision are not packed: their kernel keeps the patch data
    // uniform (the host never gives it a packed item)
    constexpr bool PACK = AMR && !(MAP && MIXED);
    const LaneStrip ls = PACK ? lane_strip(A, wk, lane) : LaneStrip{wk.patch, wk.i0, wk.r0, wk.th, 0};
    const PatchInfo pu = A.patches[PACK ? item_patch(A, wk) : wk.patch];
    const PatchInfo pi = PACK ? A.patches[ls.patch] : pu;
    ScenState *sc = &A.scen[pu.scen];
    const StepParams &P = A.P;
    if (!sc->active) return;                    // uniform over the wavefront
    const int cur = sc->cur;
    const S *qin = cur ? A.q1 : A.q0;
    S *qout = cur ? A.q0 : A.q1;
    const uint8_t *min_ = cur ? A.m1 : A.m0;
    uint8_t *mout = cur ? A.m0 : A.m1;
    const double dtd = sc->dt;
    const T dt = (T)dtd;
    const T dtdx = (T)(dtd / pu.dx), dtdy = (T)(dtd / pu.dy);
    const T tau_pre = (T)0.5 * dt;
    const T tau_post = P.splitting ? (T)0.5 * dt : dt;
    const Limiter<T> lim = limiter_of<T>(P.limiter);
    const bool trans = P.transverse == 2;

    const int sl = lane - ls.l0;                // lane within the strip
    const int col0 = ls.i0 - 2 + sl;            // its column
    int col = col0;
    if (col > pi.nx + 1) col = pi.nx + 1;       // idle lanes of a partial strip
    int fx = 0;
    const int mc = AMR ? col : map_index(col, pi.nx, pi.bc[0], pi.bc[1], &fx);
    const int xwall = col0 < 0 ? 0 : pi.nx;     // wall edge of a mapped ghost
    constexpr int D = MAP ? 2 : 0;               // x-edge family vectors: frame or global
    constexpr int DY = MAP ? 2 : 1;              // y-edge
    const long long MW = pi.nx + 4, MP = MW * (pi.ny + 4);
    const int i_hi = ls.i0 + 59 < pi.nx - 1 ? ls.i0 + 59 : pi.nx - 1;
    const bool interior = col0 >= ls.i0 && col0 <= i_hi;
    const bool interior_left = sl >= 1 && col0 - 1 >= ls.i0 && col0 - 1 <= i_hi;
    // rows of the lane's tile; the loop runs over the item's tallest tile
    // (uniform), a shorter tile's lanes idle through the rows past theirs
    const int r0 = ls.r0, th = ls.th;
    // boundary-flux recording (patch sets): lanes of the patch's edge columns
    double *ef = (AMR && pi.eoff >= 0) ? A.eflux + pi.eoff * 7 : nullptr;
    const bool e_left = ef && col == 0 && ls.i0 == 0;
    const bool e_right = ef && col0 == pi.nx && i_hi == pi.nx - 1;
    const bool e_cols = ef && interior;

    T *ring = ln.ring();
    T *base = ring + 3 * (EIG_FIELDS + (MAP ? 5 : 0)) * 64;   // mixed precision: 3 rows x 7 x 64
    // FP64 on Cartesian grids: the waves of the y-edge below and the lower
    // side of the next y-edge, each used once per row, wait in LDS between
    // rows rather than in registers the row's solves need
    constexpr bool PARK = !MIXED && !MAP;
    T *park_w = ring + 3 * EIG_FIELDS * 64, *park_s = park_w + PARK_WAVES * 64;
    int yprev_kind = 0, yside_wet = 0, yside_hyp = 0;
    Side<T> yside_prev;          // lower cell of the next y-edge (y normal frame)
    int phi_c = 0, brk_c = 0;
    // sliding windows over rows k-2 (index 0), k-1 (1) and k (2), shifted
    // down by one row at the end of each iteration.  acc[.][0] accumulates
    // the stored plane-0 variable (h, or eta' in mixed precision).
    T acc[3][7];
    int phi_w[3], brk_w[3];      // masks
    int fl_w[3] = {0, 0, 0};     // interface edge flags (patch sets)
    T b_w[3];                    // bathymetry
    T kap_w[3] = {(T)1, (T)1, (T)1};   // capacities (mapped grids)
    T qprev[7], bprev = (T)0, c2prev = (T)0, etaprev = (T)0;   // cell below (mapped y-edges)
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) qprev[m] = (T)0;
    Waves<T> yprev;              // waves of the y-edge below the new one
    T ydl[7];                    // its dot products with the edge below it
    T xtr_prev[7];               // transverse x-fluctuation entering (i, k-1)
    T bp_saved[7];               // transverse y-fluctuation entering (i, k-1) from below
    T rx = (T)0, ry = (T)0;
    double clip = 0.0;
    // error code of the lane (non-hyperbolic edge -4, non-finite result -5),
    // published once when the strip is done; nothing reads it during the step
    int errc = 0;
    bool latched = false;        // the lane latched a cell as breaking
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) { xtr_prev[m] = (T)0; bp_saved[m] = (T)0; ydl[m] = (T)0; }

    RawCell<T> nxt;
    load_raw<AMR, MAP>(pi, qin, A.bath, min_, mc, fx, r0 - 2, nxt, xwall);
    for (int j = 0; j < wk.th + 4; j++) {
        const int k = r0 - 2 + j;
        const int sk = 2, sk1 = 1, sk2 = 0;
        Cell<T> c;
        {
            RawCell<T> raw = nxt;
            mirror_raw<MAP>(raw, fx, pi.metric != nullptr);
            // issue the next row's loads before working on this one
            if (k < r0 + th + 1) load_raw<AMR, MAP>(pi, qin, A.bath, min_, mc, fx, k + 1, nxt, xwall);
            prepare_cell<T, MIXED>(P, raw, tau_pre, c, phi_c, brk_c);
            acc[sk][IH] = raw.q[IH];
            if (AMR) fl_w[sk] = (raw.mk >> 2) & 15;
        }
        phi_w[sk] = phi_c;
        brk_w[sk] = brk_c;
        b_w[sk] = c.b;
        // metric of cell (col, k): capacity, left-edge and bottom-edge frames
        T met[7] = {(T)1, (T)1, (T)0, (T)1, (T)0, (T)1, (T)1};
        if (MAP && pi.metric) {
            const double *e = pi.metric + (long long)(k + 2) * MW + (col + 2);
            HSGN_UNROLL
            for (int m = 0; m < 7; m++) met[m] = (T)e[m * MP];
        }
        kap_w[sk] = met[0];
        const T kap_l = MAP ? ln.up(met[0]) : (T)1;      // capacity of cell (col - 1, k)
        const int slot_k = (j + 4) % 3, slot_k2 = (j + 2) % 3;
        if (MIXED) {
            // increment form: the cell's state after the first source half
            // step waits in LDS while its contributions are summed from
            // zero, so that the FP32 momenta and auxiliaries are rounded
            // once per step rather than once per contribution
            HSGN_UNROLL
            for (int m = 1; m < 7; m++) {
                base[(slot_k * 7 + m) * 64 + lane] = c.q[m];
                acc[sk][m] = (T)0;
            }
        } else {
            HSGN_UNROLL
            for (int m = 1; m < 7; m++) acc[sk][m] = c.q[m];
        }

        // ---- x-edge (i-1/2, k) ----
        T xtr[7];
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) xtr[m] = (T)0;
        if (k >= r0 - 1 && k <= r0 + th) {
            Side<T> sdr, sdl;
            if (MAP) {
                T ql[7];
                HSGN_UNROLL
                for (int m = 0; m < 7; m++) ql[m] = ln.up(c.q[m]);
                const T bl = ln.up(c.b), c2l = ln.up(c.c2), etal = ln.up(c.eta);
                mapped_side(P, ql, bl, c2l, etal, met[1], met[2], (T)0 - met[2], met[1], sdl);
                mapped_side(P, c.q, c.b, c.c2, c.eta, met[1], met[2], (T)0 - met[2], met[1], sdr);
            } else {
                side_of<0>(c, sdr);
                shfl_side_up(ln, sdr, sdl);
            }
            Waves<T> xw;
            Eig<T> xe;
            // a strip's first lane has no left neighbour (its edge is a halo
            // edge, never used)
            bool ok = edge_solve<0, MIXED && FB>(ln, P, sdl, sdr, xw, xe, sl >= 1);
            errc = (!ok && sl >= 1) ? -4 : errc;
            if (MAP) set_frame(xw, xe, met[1], met[2], (T)0 - met[2], met[1], met[3]);
            Waves<T> xwl;
            shfl_waves_up<MAP>(ln, xw, xwl);
            T dl[7], dr[7];
            family_dots<D>(xwl, xw, dl);
            HSGN_UNROLL
            for (int f = 0; f < 7; f++) dr[f] = ln.dn(dl[f]);
            T F[7], am[7], ap[7];
            // mapped: dt/dx the mean of dt/(kap dx) of the edge's two cells
            const T fcx = MAP ? (T)0.5 * (dtdx / kap_l + dtdx / kap_w[sk]) : dtdx;
            correction<D>(lim, fcx, xw, dl, dr, F);
            fluctuations<0>(xw, am, ap);
            if (MAP) { to_global(xw, am); to_global(xw, ap); }
            T apc[7], amc[7], amr[7];
            HSGN_UNROLL
            for (int m = 0; m < 7; m++) { apc[m] = ap[m] - F[m]; amc[m] = am[m] + F[m]; }
            shfl_vec(ln, amc, amr, false);
            int kind_r = ln.dni(xw.kind);
            const bool zl = AMR && (fl_w[sk] & IFACE_L), zr = AMR && (fl_w[sk] & IFACE_R);
            const T ddx = MAP ? dtdx / kap_w[sk] : dtdx;
            HSGN_UNROLL
            for (int m = 0; m < 7; m++) {
                acc[sk][m] -= ddx * ((zl ? (T)0 : apc[m]) + (zr ? (T)0 : amr[m]));
                xtr[m] = (xw.kind == KIND_REGULAR ? apc[m] : (T)0)
                       + (kind_r == KIND_REGULAR ? amr[m] : (T)0);
            }
            if (AMR && k >= r0 && k < r0 + th) {
                if (e_left) {
                    HSGN_UNROLL
                    for (int m = 0; m < 7; m++) ef[(long long)k * 7 + m] = (double)amc[m];
                }
                if (e_right) {
                    HSGN_UNROLL
                    for (int m = 0; m < 7; m++)
                        ef[(long long)(pi.ny + k) * 7 + m] = -(double)apc[m];
                }
            }
            eig_store<MAP>(ring, slot_k, lane, xe);
            if (k >= r0 && k < r0 + th && (interior || interior_left)) {
                // mapped: the scaled speeds over the smaller capacity of the edge's cells
                const T kk = MAP ? tmin(kap_l, kap_w[sk]) : (T)1;
                rx = tmax(rx, tmax((T)fabs(xw.smin) / kk, tmax((T)fabs(xw.smax) / kk, (T)fabs(xw.uh) / kk)));
            }
        }

        // ---- y-edge (i, k-1/2) ----
        Side<T> yside;
        side_of<1>(c, yside);
        if (k >= r0 - 1) {
            // the x-edge eigenstructure of row k-2 read from LDS ahead of the
            // y-edge solve, whose arithmetic hides the latency (the parked
            // waves are read after it: held through the solve, they would
            // cost more registers than the wait)
            Eig<T> exk2;
            eig_load<MAP>(ring, slot_k2, lane, exk2);
            Waves<T> yw;
            Eig<T> ye;
            bool ok;
            if (MAP) {
                // frame of the bottom edge of cell (i, k): tangent (n_y, -n_x)
                Side<T> ysl, ysr;
                mapped_side(P, qprev, bprev, c2prev, etaprev, met[4], met[5], met[5], (T)0 - met[4], ysl);
                mapped_side(P, c.q, c.b, c.c2, c.eta, met[4], met[5], met[5], (T)0 - met[4], ysr);
                ok = edge_solve<0, MIXED && FB>(ln, P, ysl, ysr, yw, ye);
                set_frame(yw, ye, met[4], met[5], met[5], (T)0 - met[4], met[6]);
            } else if constexpr (PARK) {
                Side<T> ysl;
                unpark_side(park_s, lane, yside_wet, yside_hyp, ysl);
                ok = edge_solve<1, MIXED && FB>(ln, P, ysl, yside, yw, ye);
            } else {
                ok = edge_solve<1, MIXED && FB>(ln, P, yside_prev, yside, yw, ye);
            }
            // (a lane past its tile's rows solves its last row against itself)
            errc = (!ok && k <= r0 + th + 1) ? -4 : errc;
            if (k >= r0 && k <= r0 + th && interior) {
                const T kk = MAP ? tmin(kap_w[sk1], kap_w[sk]) : (T)1;
                ry = tmax(ry, tmax((T)fabs(yw.smin) / kk, tmax((T)fabs(yw.smax) / kk, (T)fabs(yw.uh) / kk)));
            }
            if (k >= r0) {
                if constexpr (PARK) unpark_waves(park_w, lane, yprev_kind, yprev);
                T dk[7];
                family_dots<DY>(yw, yprev, dk);
                if (k - 1 >= r0 && k - 1 <= r0 + th) {
                    // the y-edge (i, k-3/2) between rows k-2 and k-1 is complete
                    T G[7], bm[7], bp[7];
                    const T fcy = MAP ? (T)0.5 * (dtdy / kap_w[sk2] + dtdy / kap_w[sk1]) : dtdy;
                    correction<DY>(lim, fcy, yprev, ydl, dk, G);
                    if (MAP) {
                        fluctuations<0>(yprev, bm, bp);
                        to_global(yprev, bm);
                        to_global(yprev, bp);
                    } else {
                        fluctuations<1>(yprev, bm, bp);
                    }
                    T btm[7], btp[7];
                    const bool zb = AMR && (fl_w[sk1] & IFACE_B), zt = AMR && (fl_w[sk2] & IFACE_T);
                    HSGN_UNROLL
                    for (int m = 0; m < 7; m++) {
                        T bpc = bp[m] - G[m], bmc = bm[m] + G[m];
                        acc[sk1][m] -= (MAP ? dtdy / kap_w[sk1] : dtdy) * (zb ? (T)0 : bpc);
                        acc[sk2][m] -= (MAP ? dtdy / kap_w[sk2] : dtdy) * (zt ? (T)0 : bmc);
                        btp[m] = yprev.kind == KIND_REGULAR ? bpc : (T)0;
                        btm[m] = yprev.kind == KIND_REGULAR ? bmc : (T)0;
                    }
                    if (AMR && e_cols) {
                        // the y-edge between rows k-2 and k-1
                        if (k - 1 == 0) {
                            HSGN_UNROLL
                            for (int m = 0; m < 7; m++) {
                                double *e = ef + (long long)(2 * pi.ny + col) * 7 + m;
                                *e = (double)(bm[m] + G[m]) + *e;
                            }
                        }
                        if (k - 1 == pi.ny) {
                            HSGN_UNROLL
                            for (int m = 0; m < 7; m++) {
                                double *e = ef + (long long)(2 * pi.ny + pi.nx + col) * 7 + m;
                                *e = -(double)(bp[m] - G[m]) + *e;
                            }
                        }
                    }
                    if (k - 2 >= r0 && k - 2 <= r0 + th - 1) {
                        // transverse y-fluctuation entering (i, k-2), split by
                        // the x-edges (i-1/2, k-2) and (i+1/2, k-2)
                        T ytr[7], ytl[7];
                        HSGN_UNROLL
                        for (int m = 0; m < 7; m++) ytr[m] = bp_saved[m] + btm[m];
                        shfl_vec(ln, ytr, ytl, true);
                        T Ft[7];
                        HSGN_UNROLL
                        for (int m = 0; m < 7; m++) Ft[m] = (T)0;
                        const T kap2_l = MAP ? ln.up(kap_w[sk2]) : (T)1;   // cell (i - 1, k - 2)
                        if (trans && exk2.wet) {
                            T vp[7], vm[7];
                            trans_split<D>(exk2, ytl, 1, vp);
                            trans_split<D>(exk2, ytr, -1, vm);
                            if (MAP) {
                                // each part weighted by the edge's length ratio over
                                // the capacity of the cell it entered
                                const T wa = exk2.gm / kap2_l, wb = exk2.gm / kap_w[sk2];
                                HSGN_UNROLL
                                for (int m = 0; m < 7; m++)
                                    Ft[m] = (T)-0.5 * dtdy * (wa * vp[m] + wb * vm[m]);
                            } else {
                                HSGN_UNROLL
                                for (int m = 0; m < 7; m++) Ft[m] = (T)-0.5 * dtdy * (vp[m] + vm[m]);
                            }
                        }
                        T Ftr[7];
                        shfl_vec(ln, Ft, Ftr, false);
                        const bool fzl = AMR && (fl_w[sk2] & IFACE_L);
                        const bool fzr = AMR && (fl_w[sk2] & IFACE_R);
                        const T ddx2 = MAP ? dtdx / kap_w[sk2] : dtdx;
                        HSGN_UNROLL
                        for (int m = 0; m < 7; m++)
                            acc[sk2][m] -= ddx2 * ((fzr ? (T)0 : Ftr[m]) - (fzl ? (T)0 : Ft[m]));
                        if (AMR && (e_left || e_right)) {
                            long long e0 = (long long)((e_left ? 0 : pi.ny) + (k - 2)) * 7;
                            HSGN_UNROLL
                            for (int m = 0; m < 7; m++) ef[e0 + m] = ef[e0 + m] + (double)Ft[m];
                        }
                    }
                    HSGN_UNROLL
                    for (int m = 0; m < 7; m++) bp_saved[m] = btp[m];
                }
                HSGN_UNROLL
                for (int f = 0; f < 7; f++) ydl[f] = dk[f];
            }
            T Gt[7];
            HSGN_UNROLL
            for (int m = 0; m < 7; m++) Gt[m] = (T)0;
            if (trans && k >= r0 && k <= r0 + th && ye.wet) {
                // transverse x-fluctuations entering (i, k-1) [up] and (i, k) [down]
                T vp[7], vm[7];
                trans_split<DY>(ye, xtr_prev, 1, vp);
                trans_split<DY>(ye, xtr, -1, vm);
                const bool zt = AMR && (fl_w[sk1] & IFACE_T), zb = AMR && (fl_w[sk] & IFACE_B);
                const T wa = MAP ? ye.gm / kap_w[sk1] : (T)1, wb = MAP ? ye.gm / kap_w[sk] : (T)1;
                const T ddy1 = MAP ? dtdy / kap_w[sk1] : dtdy, ddy0 = MAP ? dtdy / kap_w[sk] : dtdy;
                HSGN_UNROLL
                for (int m = 0; m < 7; m++) {
                    Gt[m] = MAP ? (T)-0.5 * dtdx * (wa * vp[m] + wb * vm[m])
                                : (T)-0.5 * dtdx * (vp[m] + vm[m]);
                    acc[sk1][m] -= ddy1 * (zt ? (T)0 : Gt[m]);
                    acc[sk][m] += ddy0 * (zb ? (T)0 : Gt[m]);
                }
            }
            if (AMR && e_cols && (k == 0 || k == pi.ny) && k >= r0 && k <= r0 + th) {
                // transverse part of the patch's lower or upper boundary edge
                long long e0 = (long long)(k == 0 ? 2 * pi.ny + col : 2 * pi.ny + pi.nx + col) * 7;
                HSGN_UNROLL
                for (int m = 0; m < 7; m++) ef[e0 + m] = (double)Gt[m];
            }
            if constexpr (PARK) {
                park_waves(park_w, lane, yw);
                yprev_kind = yw.kind;
            } else {
                yprev = yw;
            }
        }

        // ---- row k-2 complete: second source half step and fix-ups ----
        if (k - 2 >= r0 && k - 2 <= r0 + th - 1) {
            int phi = phi_w[sk2], brk = brk_w[sk2];
            int swe = !phi || brk;
            T bb = b_w[sk2];
            T c2 = swe ? (T)0 : (T)P.a2g * still_depth(P, bb) + (T)P.c2f;
            // depth in the compute type for the source step
            T qn[7];
            HSGN_UNROLL
            for (int m = 0; m < 7; m++)
                qn[m] = (MIXED && m > 0) ? base[(slot_k2 * 7 + m) * 64 + lane] + acc[sk2][m]
                                         : acc[sk2][m];
            qn[IH] = depth_of<T, MIXED>(P, acc[sk2][IH], bb);
            source_or_clear(P, qn, c2, swe, tau_post);
            // sponge: every variable relaxed towards the state at rest by an
            // implicit Euler step (FP64: h towards H; mixed precision: eta'
            // towards its rest value (b - eta0)^+)
            if (SP && pi.sp_rate > 0.0) {               // uniform over the wavefront
                const double sg = sponge_sigma(pi, col0, k - 2);
                if (sg > 0.0) {
                    const double f = 1.0 / (1.0 + dtd * sg);
                    if constexpr (MIXED) {
                        const T fT = (T)f;
                        const T er = tmax((T)0, bb - (T)P.eta0);
                        acc[sk2][IH] = er + (acc[sk2][IH] - er) * fT;
                        HSGN_UNROLL
                        for (int m = 1; m < 7; m++) qn[m] = qn[m] * fT;
                    } else {
                        const double H = still_depth(P, (double)bb);
                        acc[sk2][IH] = (T)(H + ((double)acc[sk2][IH] - H) * f);
                        HSGN_UNROLL
                        for (int m = 1; m < 7; m++) qn[m] = (T)((double)qn[m] * f);
                    }
                }
            }
            // fix-ups: clipping (the clipped mass summed in FP64), dry cells,
            // breaking latch (eta - eta0 > kappa H), SWE cells.  FP64: on h
            // as the oracle does; mixed precision: on the stored deviation
            // eta' directly, in FP64 for SWE cells (phi_T = 0 or breaking:
            // every dry and shallow cell, whose edges are solved in FP64 too)
            // and in FP32 for the others.  The kernel without the FP64 edge
            // solve (FB false) holds no SWE cell.
            S out0;
            S qs[7];
            bool bad;
            if constexpr (MIXED) {
                T eta = acc[sk2][IH];
                bool dry;
                if (FB && swe) {
                    double etaD = (double)eta;
                    const double bD = (double)bb;
                    const double hD = (etaD + P.eta0) - bD;
                    if (hD < 0.0) {
                        clip += MAP ? -hD * (double)kap_w[sk2] * pu.dx * pu.dy
                                    : -hD * pu.dx * pu.dy;
                        etaD = bD - P.eta0;
                    }
                    dry = !(hD > P.dry_tol);
                    eta = (T)etaD;
                } else {
                    T h = eta + (T)P.eta0 - bb;
                    if (h < (T)0) {
                        clip += MAP ? -(double)h * (double)kap_w[sk2] * pu.dx * pu.dy
                                    : -(double)h * pu.dx * pu.dy;
                        h = (T)0;
                        eta = bb - (T)P.eta0;
                    }
                    dry = !(h > (T)P.dry_tol);
                }
                if (dry) {
                    HSGN_UNROLL
                    for (int m = 1; m < 7; m++) qn[m] = (T)0;
                } else if (P.kappa > 0.0 && phi && !brk) {
                    T H = tmax((T)P.eta0 - bb, (T)0);
                    if (eta > (T)P.kappa * H) {
                        brk = 1;
                        latched = interior;
                    }
                }
                if (!phi || brk || dry) {
                    qn[IHW] = (T)0; qn[IHS] = (T)0; qn[IHP] = (T)0; qn[IHPB] = (T)0;
                }
                out0 = (S)eta;
                bad = !finite_val<T>(eta);
                HSGN_UNROLL
                for (int m = 1; m < 7; m++) { qs[m] = (S)qn[m]; bad = bad || !finite_val<T>(qn[m]); }
            } else {
                double hD = (double)acc[sk2][IH];
                double qd[7];
                HSGN_UNROLL
                for (int m = 1; m < 7; m++) qd[m] = (double)qn[m];
                if (hD < 0.0) {
                    clip += MAP ? -hD * (double)kap_w[sk2] * pu.dx * pu.dy : -hD * pu.dx * pu.dy;
                    hD = 0.0;
                }
                if (hD <= P.dry_tol) {
                    HSGN_UNROLL
                    for (int m = 1; m < 7; m++) qd[m] = 0.0;
                } else if (P.kappa > 0.0 && phi && !brk) {
                    double bD = (double)bb;
                    double H = P.eta0 - bD;
                    H = H > 0.0 ? H : 0.0;
                    if (hD + bD - P.eta0 > P.kappa * H) brk = 1;
                }
                if (!phi || brk || hD <= P.dry_tol) {
                    qd[IHW] = 0.0; qd[IHS] = 0.0; qd[IHP] = 0.0; qd[IHPB] = 0.0;
                }
                out0 = (S)hD;
                bad = !finite_val<double>(hD);
                HSGN_UNROLL
                for (int m = 1; m < 7; m++) { qs[m] = (S)qd[m]; bad = bad || !finite_val<double>(qd[m]); }
            }
            errc = (interior && bad) ? -5 : errc;
            if (interior) {
                long long idx = (long long)(k - 2) * pi.pitch + col0;
                long long plane = pi.plane;
                S *qo = qout + pi.qoff + idx;
                qo[0] = out0;
                HSGN_UNROLL
                for (int m = 1; m < 7; m++) qo[m * plane] = qs[m];
                mout[pi.coff + idx] = (uint8_t)(phi | (brk << 1) | (AMR ? fl_w[sk2] << 2 : 0));
            }
        }
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) {
            xtr_prev[m] = xtr[m];
            acc[0][m] = acc[1][m];
            acc[1][m] = acc[2][m];
            if (MAP) qprev[m] = c.q[m];
        }
        if (MAP) {
            bprev = c.b; c2prev = c.c2; etaprev = c.eta;
            kap_w[0] = kap_w[1]; kap_w[1] = kap_w[2];
        }
        phi_w[0] = phi_w[1]; phi_w[1] = phi_w[2];
        fl_w[0] = fl_w[1]; fl_w[1] = fl_w[2];
        brk_w[0] = brk_w[1]; brk_w[1] = brk_w[2];
        b_w[0] = b_w[1]; b_w[1] = b_w[2];
        if constexpr (PARK) {
            park_side(park_s, lane, yside);
            yside_wet = yside.wet;
            yside_hyp = yside.hyp;
        } else {
            yside_prev = yside;
        }
    }
    if (errc) sc->err = errc;
    if (MIXED && A.latch && ln.any(latched) && lane == 0) *A.latch = 1;
    ln.finish(A, wid, pu.scen, (double)rx, (double)ry, clip);
}

}  // namespace hsgn
