// hsgn_amr.hpp -- tables and kernel launchers of static patch sets (AMR).
//
// A scenario with more than one patch is a patch set: levels 0..L-1 with
// refinement ratio 4 in space and time, every patch stored with a 2-cell
// ghost frame.  The host builds, once, the tables below; the kernels that
// use them run between the step launches of the levels:
//   ghost fill   copy from the same-level patch covering a ghost cell (or,
//                on level 0, from the domain cell a boundary condition maps
//                it to); otherwise coarse-to-fine interpolation, linear in
//                time between the coarse old and new states and linear in
//                space with minmod-limited slopes of eta' and the momenta
//                and auxiliaries;
//   flux sums    after every fine substep, per fine boundary edge facing the
//                coarse level: R += E + (+/-) dflux(C*, g*), E being what the
//                fine step sent through the edge and dflux the total
//                fluctuation between the coarse cell and the fine ghost after
//                their first source half steps;
//   reflux       after the substeps, the coarse cell next to the fine patch
//                takes -/+ dt/dx times the mean of the 4 x 4 fine records
//                over its edge (its own contribution through that edge was
//                left out of its step), then the cell fix-ups;
//   average-down covered coarse cells take the mean of their 4 x 4 cells.
// The wave-propagation AMR of Berger and LeVeque, cited in Sec. 4, is the
// model; the rules above are the precise form implemented.
//
// Mapped patch sets (Sec. 4, mapped grids; every patch has a metric): the
// fine nodes are the bilinear refinement of the coarse ones (the caller's
// rule), ghost interpolation stays in index space, a level-0 wall ghost
// mirrors the momentum about the wall edge's unit normal, the flux records
// take the total fluctuation solved in the fine edge's frame and scaled by
// its length ratio, refluxing divides by the coarse capacity and averaging
// down takes sum(kap q) / sum(kap) over the 4 x 4 fine cells.
#pragma once

#include <hip/hip_runtime.h>

#include "hsgn_march.hpp"

namespace hsgn {

constexpr int AMR_RATIO = 4;

// "local" = j * pitch + i relative to the patch's interior cell (0, 0);
// negative or beyond nx for ghost cells
struct GhostCopy {
    int dp, dl;          // destination patch, local
    int sp, sl;          // source patch, local
    int flips;           // bit 0: negate hu, bit 1: negate hv (walls)
    int wx, wy;          // mapped walls: source-patch local of the cell whose
                         // left (bit 0) / bottom (bit 1) edge is the wall
};

struct GhostInterp {
    int dp, dl;
    int cp[5], cl[5];    // coarse centre, left, right, below, above (cp < 0: none)
    float ox, oy;        // offset of the ghost centre in coarse cells (+-1/8, +-3/8)
};

struct FluxRec {
    int fp, entry;       // fine patch, boundary-edge entry
    int gl;              // the fine ghost cell outside the edge
    int cp, cl;          // the coarse cell containing it
    int dir, low;        // 0 x / 1 y; low = the coarse cell is left of / below the edge
};

struct RefluxRec {
    int cp, cl;          // coarse cell
    int fp[4], e0[4];    // per edge L, R, B, T: fine patch (or -1), first entry
};

struct AvgRec {
    int fp, fl;          // fine patch, local of the lower-left fine cell
    int cp, cl;          // coarse cell
};

template <class S>
struct AmrBuffers {
    const PatchInfo *patches;
    const ScenState *scen;
    S *q0, *q1;
    S *bath;
    uint8_t *m0, *m1;
};

// launchers (hsgn_amr.hip); every kernel skips work of scenarios in error
void launch_halo_copy64(const AmrBuffers<double> &B, const GhostCopy *r, int n, hipStream_t s);
void launch_halo_copy32(const AmrBuffers<float> &B, const GhostCopy *r, int n, hipStream_t s);
void launch_halo_interp64(const AmrBuffers<double> &B, const GhostInterp *r, int n, double theta,
                          double eta0, double dry_tol, hipStream_t s);
void launch_halo_interp32(const AmrBuffers<float> &B, const GhostInterp *r, int n, double theta,
                          double eta0, double dry_tol, hipStream_t s);
void launch_ghost_bath64(const AmrBuffers<double> &B, const GhostCopy *c, int nc,
                         const GhostInterp *r, int ni, hipStream_t s);
void launch_ghost_bath32(const AmrBuffers<float> &B, const GhostCopy *c, int nc,
                         const GhostInterp *r, int ni, hipStream_t s);
void launch_avgdown64(const AmrBuffers<double> &B, const AvgRec *r, int n, bool bath_only,
                      hipStream_t s);
// keep: per patch, 1 where a bathymetry-only average-down keeps the
// covered cells' depth (mixed storage of eta'); null keeps eta'
void launch_avgdown32(const AmrBuffers<float> &B, const AvgRec *r, int n, bool bath_only,
                      hipStream_t s, const uint8_t *keep = nullptr);
void launch_bflux64(const AmrBuffers<double> &B, const StepParams &P, const FluxRec *r, int n,
                    const double *E, double *R, hipStream_t s);
void launch_bflux32(const AmrBuffers<float> &B, const StepParams &P, const FluxRec *r, int n,
                    const double *E, double *R, hipStream_t s);
void launch_reflux64(const AmrBuffers<double> &B, const StepParams &P, const RefluxRec *r, int n,
                     const double *R, double *rclip, hipStream_t s);
void launch_reflux32(const AmrBuffers<float> &B, const StepParams &P, const RefluxRec *r, int n,
                     const double *R, double *rclip, hipStream_t s);
void launch_iface(const PatchInfo *patches, const RefluxRec *r, int n, uint8_t *m0, uint8_t *m1,
                  hipStream_t s);
void launch_fill_zero(double *p, long long n, hipStream_t s);

// regridding (hsgn_regrid): a rectangle of interior cells copied from a patch
// of the old storage (buffers sq, sb, sm: the ones holding its current step)
// to a patch of the new storage, and a new patch filled from its coarse
// parent.  Records are laid end to end: c0 is the first cell of a record in
// the launch.
template <class S>
struct RegridCopy {
    PatchInfo src, dst;
    const S *sq;
    const S *sb;
    const uint8_t *sm;
    int si0, sj0, di0, dj0;   // rectangle origin, interior cells of each patch
    int nx, ny;
    long long c0;
};

struct RegridInterp {
    PatchInfo fine, coarse;   // both in the new storage
    int ci0, cj0;             // coarse-local cell under the fine cell (0, 0)
    int pad;
    long long c0;
};

// bathymetry from the level-0 bathymetry B0[NY][NX] (cell-centred): the
// bilinear interpolant at the centres of a level-`level` patch whose cell
// (0, 0) is level cell (I0, J0); at level 0 it returns B0 itself
struct TopoRec {
    PatchInfo p;
    int I0, J0, level, pad;
    long long c0;
};
void launch_topo64(const TopoRec *r, int nr, long long total, const double *B0, int NX, int NY,
                   double *bath, hipStream_t s);
void launch_topo32(const TopoRec *r, int nr, long long total, const double *B0, int NX, int NY,
                   float *bath, hipStream_t s);

// the flags of the level-l patches of one regrid, in one launch: a record
// per patch, its flags laid end to end in the output (c0: its first flag)
struct FlagRec {
    PatchInfo p;
    long long c0;
};
void launch_regrid_flag64(const FlagRec *r, int nr, long long total, const double *q,
                          const double *bath, uint8_t *out, double eta0, double dry_tol,
                          double tol, hipStream_t s);
void launch_regrid_flag32(const FlagRec *r, int nr, long long total, const float *q,
                          const float *bath, uint8_t *out, double eta0, double dry_tol,
                          double tol, hipStream_t s);
void launch_regrid_copy64(const RegridCopy<double> *r, int nr, long long total, double *q,
                          const double *bath, uint8_t *m0, uint8_t *m1, double eta0,
                          double dry_tol, hipStream_t s);
void launch_regrid_copy32(const RegridCopy<float> *r, int nr, long long total, float *q,
                          const float *bath, uint8_t *m0, uint8_t *m1, double eta0,
                          double dry_tol, hipStream_t s);
void launch_regrid_interp64(const RegridInterp *r, int nr, long long total, double *q,
                            const double *bath, uint8_t *m0, uint8_t *m1, double eta0,
                            double dry_tol, hipStream_t s);
void launch_regrid_interp32(const RegridInterp *r, int nr, long long total, float *q,
                            const float *bath, uint8_t *m0, uint8_t *m1, double eta0,
                            double dry_tol, hipStream_t s);

}  // namespace hsgn
