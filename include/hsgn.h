/*
 * hsgn.h -- C ABI of the MI355X time-step library for the hyperbolic
 * Serre-Green-Naghdi system coupled to the shallow water equations.
 *
 * The library advances sets of 2D Cartesian grid patches by the explicit
 * finite-volume step of Sec. 4 of the paper: per-edge f-wave Riemann solves
 * (eq. total fluctuation, Appendix C eigenstructure, Einfeldt speeds) with
 * limited second-order and transverse corrections, the flux-difference
 * cell update, the SDIRK(2,2) relaxation source step (Strang or Lie
 * splitting), and the cell-wise switch to the shallow water equations where
 * the still-water depth within one cell is below h_star (eq. transition
 * function, c^2 = alpha^2 g H phi_T) or where a cell is latched as breaking.
 * The time step follows the CFL condition with the global maximum wave speed
 * (Sec. 4).  All arithmetic runs in HIP kernels on the device.
 *
 * Conventions
 *   - Every call returns an int status: HSGN_OK (0) or a negative HSGN_E*
 *     code.  No call throws, aborts or prints.  hsgn_last_error() gives a
 *     context-owned message for the last failure.
 *   - State arrays at this interface are float64, layout q[7][ny][nx]
 *     (row-major, x fastest), conserved variables in the order h, hu, hv,
 *     hw, h*sigma, hp, h*p_b (Appendix C).  Bathymetry b[ny][nx] is float64,
 *     measured from the sea level eta0 (negative below it).
 *   - Pointers passed in are borrowed for the duration of the call only
 *     (copy semantics); on_device = 1 means the pointer is device memory on
 *     the context's device, 0 means host memory.
 *   - All device work is enqueued on the stream given to hsgn_create (a
 *     borrowed hipStream_t; NULL = the default stream), mixed-precision
 *     steps partly on a second stream joined back into it (hsgn_create).
 *   - A context owns its device buffers: two state buffers (the step reads
 *     one and writes the other), bathymetry, two mask buffers, per-scenario
 *     clocks and gauge records.  Its patch-set tables (ghost cells, boundary
 *     fluxes, covered cells; 16 to 56 bytes per record) are kept in pinned
 *     host memory too, or ordinary memory where pinning fails.
 *   - Calls on one context must not overlap; calls on different contexts
 *     may come from different host threads.  hsgn_finalize and hsgn_regrid
 *     build and check their tables on a shared set of host worker threads
 *     (at most 16, made on first use); such calls from several threads take
 *     turns for them.
 *   - A scenario is an independent simulation with its own clock and time
 *     step; each patch belongs to one scenario.
 *   - Patch sets (static AMR, the block-structured refinement of Sec. 4): a
 *     scenario with more than one patch.  Level-0 patches tile a rectangle
 *     (the domain; their boundary conditions apply on its sides, so they
 *     must agree); level-l patches have spacing dx0 / 4^l, corners on
 *     level-(l-1) cell corners, sides that are multiples of 4, stay one
 *     level-(l-1) cell inside the domain and lie in the union of level-(l-1)
 *     patches with one level-(l-1) cell to spare.  Patches of one level do
 *     not overlap.  Each level-0 step runs 4 substeps of every level-1
 *     patch, each of which runs 4 level-2 substeps, and so on.  Ghost cells
 *     come from the same-level neighbour or the domain boundary condition,
 *     else from the coarser level: linear in time between its old and new
 *     states, linear in space with minmod-limited slopes of eta' = h + b -
 *     eta0, hu, hv, hw, h sigma, hp, h p_b (zero slopes next to dry cells).
 *     Coarse cells next to a finer patch take the finer patch's fluxes
 *     (refluxing: their own contribution through that edge is replaced by
 *     the mean of the 4 x 4 fine-edge, fine-substep fluxes, which keeps the
 *     mass exact); covered coarse cells take the mean of their 4 x 4 fine
 *     cells after the substeps, and their bathymetry the mean of the fine
 *     bathymetry.  Patch sets advance with fixed steps only.
 */
#ifndef HSGN_H
#define HSGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSGN_OK          0
#define HSGN_EINVAL     -1   /* bad argument or call order */
#define HSGN_ENOMEM     -2   /* device or host allocation failed */
#define HSGN_ECFL       -3   /* fixed step exceeded cfl_max (state kept at last good step) */
#define HSGN_ENONHYP    -4   /* g h + p + c^2 <= 0 at an edge (Sec. 3 hyperbolicity) */
#define HSGN_ENAN       -5   /* non-finite value produced */
#define HSGN_ERANGE     -6   /* gauge outside its scenario's patches */
#define HSGN_EDEVICE    -7   /* HIP runtime error */
#define HSGN_ENOTSUP    -8   /* option not supported by this build */
#define HSGN_ESCRATCH   -9   /* grid larger than hsgn_advance_static's working memory */

#define HSGN_BC_PERIODIC 0
#define HSGN_BC_WALL     1   /* reflecting wall: mirror, normal momentum negated */
#define HSGN_BC_EXTRAP   2   /* zeroth-order extrapolation */

typedef struct hsgn_params {
    int model;          /* 0 = HSGN (eq. HSGN, 7 variables); 1 = mbHSGN (eq.
                           mbHSGN: the same 7-plane layout with h sigma and
                           h p_b identically zero, which the library keeps) */
    int precision;      /* 0 = FP64; 1 = mixed: FP32 storage of eta' = h + b -
                           eta0 and FP32 arithmetic, FP64 for every edge with
                           an SWE or dry side, for cell fix-ups and mass sums */
    double g;           /* gravity */
    double alpha;       /* relaxation parameter alpha = c / sqrt(g H), Sec. 3 */
    double eta0;        /* sea level at rest */
    double h_star;      /* SWE transition depth of phi_T */
    double dry_tol;     /* cells with h <= dry_tol are dry */
    double xi0, xi1;    /* bathymetry sharpness sensor parameters (Sec. 4) */
    double cfl;         /* Courant number targeted by the adaptive step */
    double cfl_max;     /* largest accepted Courant number */
    double kappa;       /* breaking latch eta - eta0 > kappa H; <= 0 disables */
    int nbr_n;          /* neighbourhood half-width n of phi_T (0..2) */
    int limiter;        /* 0 first order, 1 minmod, 2 MC, 3 unlimited */
    int transverse;     /* 0 none, 2 transverse waves incl. corrections */
    int splitting;      /* 0 Lie, 1 Strang */
    int tile_rows;      /* rows per marching tile; <= 0 lets the library choose */
    double c2;          /* 0: c^2 = alpha^2 g H phi_T (Sec. 3.3); > 0: this fixed
                           relaxation parameter c^2 (m^2/s^2) times phi_T, as in
                           the steady-state tests of Sec. 5; negative or NaN
                           is HSGN_EINVAL */
} hsgn_params;

typedef struct hsgn_diag {
    double mass;            /* sum of h dx dy (FP64, fixed summation order) */
    double clipped_mass;    /* water added by clipping negative depths */
    double max_courant;     /* largest accepted Courant number so far */
    double last_courant;    /* Courant number of the last accepted step */
    long long steps;        /* accepted steps */
    long long rejected;     /* rejected adaptive attempts */
    long long cell_updates; /* interior cell updates of accepted steps */
    long long n_swe_cells;  /* cells with phi_T = 0 or latched breaking */
    long long n_breaking;   /* cells latched as breaking */
} hsgn_diag;

typedef struct hsgn_ctx hsgn_ctx;

/* Create a context.  *p is copied.  hip_stream: borrowed hipStream_t.
 * Mixed precision (precision 1) splits each step launch: the work items
 * are classified from the step's input mask, the items that cannot need the
 * FP64 near-shore solve run a kernel without it, and the others run the full
 * kernel on a second stream the context owns (default priority), forked
 * from and joined back into hip_stream with events, so that work enqueued on
 * hip_stream after a call still follows the whole step.  The two kernels
 * compute the same method in the same order; being two instantiations, they
 * can round an FP32 operation differently in a few cells (the compiler fuses
 * products into sums per instantiation).  The environment variable
 * HSGN_NO_KERNEL_SPLIT=1, read here, runs the full kernel on every item (a
 * diagnostic).  Within an advance over single grids only, the items are
 * classified again only after a step latched a cell as breaking.
 * Patch sets pack column strips narrower than 60 cells, up to four of one
 * refinement level, into one wavefront's work item (mapped patch sets in
 * mixed precision excepted); HSGN_NO_PACKING=1, read here, gives every
 * strip its own (a diagnostic: the state is the same bit for bit).
 * HSGN_PAGEABLE_TABLES=1, read whenever a table grows, keeps the patch-set
 * tables in ordinary host memory instead of pinned memory (a diagnostic).
 * Errors: EINVAL (bad parameters), ENOTSUP (model/precision), EDEVICE. */
int hsgn_create(const hsgn_params *p, void *hip_stream, hsgn_ctx **out);

/* Add an nx x ny patch of refinement level `level` (0 = coarsest, at most
 * 5) with cell size dx, dy and lower-left corner (x0, y0) to a scenario
 * (scenarios are numbered from 0 and need not be declared).  bc[4] =
 * {x-low, x-high, y-low, y-high}; periodic sides come in pairs.
 * Errors: EINVAL (nx or ny < 4, bad bc, after finalize). */
int hsgn_add_grid(hsgn_ctx *c, int scenario, int level, int nx, int ny, double x0, double y0,
                  double dx, double dy, const int bc[4], int *patch_id);

/* Check the patch sets (rules above), allocate the device buffers and build
 * the work and patch-set tables.  Errors: EINVAL (with the broken rule in
 * hsgn_last_error), ENOMEM. */
int hsgn_finalize(hsgn_ctx *c);

/* Bathymetry b[ny][nx] of a patch; computes H = (eta0 - b)^+ and phi_T (the
 * minimum of H over the (2n+1)^2 box through the boundary map exceeds
 * h_star) and clears the breaking latch.  A state already set keeps each
 * cell's depth h under the new bottom in both precisions, so that the
 * surface moves with it: called between steps, this is the sea-floor motion
 * that generates the Tohoku tsunami of Sec. 6.4 (covered cells of a coarser
 * level keep theirs too when their bathymetry is averaged anew).  The library
 * keeps a host copy of b (8 bytes per cell; regridding rebuilds from it); a
 * device pointer is read with a synchronous copy. */
int hsgn_set_bathymetry(hsgn_ctx *c, int patch, const double *b, int on_device);

/* Sponge layer of a scenario (the relaxation sponge of the Tohoku case,
 * Sec. 6.4, where it is cited without a description; this is a reading):
 * within width[e] metres of the domain side e (0 x-low, 1 x-high, 2 y-low,
 * 3 y-high; 0 = none) every conserved variable of a cell is relaxed towards
 * the state at rest (h = H = (eta0 - b)^+, the others zero) once per step,
 * after the second source half step and before the fix-ups, by the implicit
 * Euler factor 1 / (1 + dt sigma), sigma = rate ((w - d) / w)^2 with d the
 * distance of the cell centre from that side (the largest over the sides).
 * The domain is the grid, or for a patch set the rectangle its level-0
 * patches tile; every patch of the scenario follows it, and regridding
 * keeps it.  rate = 0 removes the sponge.  After hsgn_finalize.
 * Errors: EINVAL (no such scenario, negative or non-finite width or rate). */
int hsgn_set_sponge(hsgn_ctx *c, int scenario, const double width[4], double rate);

/* Mapped grid (Sec. 4, mapped grids): makes patch `patch` (a single grid or
 * a patch of a patch set) a planar, logically rectangular mapped grid.  xn,
 * yn (host, row-major,
 * [ny + 5][nx + 5], copied) are the coordinates of nodes (i, j) for
 * i = -2..nx+2, j = -2..ny+2 at [j + 2][i + 2], the two ghost layers
 * included; cell (i, j) has corners (i, j), (i+1, j), (i+1, j+1), (i, j+1)
 * counter-clockwise.  The patch's dx, dy become the computational spacings:
 * a cell's capacity is its area over dx dy, an edge's length ratio its length
 * over dy (edges between columns) or dx (edges between rows).  Each edge's
 * Riemann problem is solved in the frame of its unit normal; waves, speeds
 * and fluctuations are rotated back and scaled by the length ratio, and
 * updates are divided by the capacity.  Momenta (hu, hv) and the state stay
 * in the physical frame; walls mirror the momentum about the wall edge.
 * Gauges and the sponge layer use computational coordinates.  Mass in
 * hsgn_diagnostics is sum(capacity h) dx dy.
 * Patch sets: every patch of the set takes a mapping before the next
 * hsgn_advance, or none does (else that call fails with HSGN_EINVAL).  The
 * caller gives each patch the nodes of its frame; for the refluxing and
 * averaging down to conserve the capacity-weighted mass, a finer patch's
 * nodes must be the bilinear refinement of the coarser level's (its cells
 * then tile each coarse cell exactly).  Ghost interpolation from the coarser
 * level stays in index space; level-0 walls mirror the momentum about the
 * wall edge; the coarse-fine flux records are solved in each fine edge's
 * frame; refluxing divides by the coarse capacity, and averaging down takes
 * sum(capacity q) / sum(capacity) over the 4 x 4 fine cells (the bathymetry
 * likewise, recomputed at the next hsgn_advance).
 * After hsgn_finalize; may be called again to change the mapping.
 * The first mapped single grid (patch-set patch) in a context drops a
 * captured step graph: the single-grid (patch-set) step launches switch to
 * the mapped kernel.  HSGN_ENOTSUP: a context with a sponge layer.
 * HSGN_EINVAL: bad patch, null pointers, or a cell of non-positive area or an
 * edge of zero length (the patch keeps its previous geometry). */
int hsgn_set_mapping(hsgn_ctx *ctx, int patch, const double *xn, const double *yn);

/* State q[7][ny][nx] (float64) of a patch, copied in or out: the conserved
 * variables of eq. HSGN (Sec. 3) in the order of the eigenstructure of
 * Appendix C (h, hu, hv, hw, h sigma, hp, h p_b).  Mixed precision stores
 * eta' and converts on the way in and out.  A device pointer is copied with a synchronous copy.  Errors: EINVAL
 * (bad patch, null pointer, before finalize). */
int hsgn_set_state(hsgn_ctx *c, int patch, const double *q, int on_device);
int hsgn_get_state(hsgn_ctx *c, int patch, double *q, int on_device);

/* Mask byte per cell: bit0 = phi_T (eq. transition: dispersive where the
 * still-water depth exceeds h_star), bit1 = the breaking latch of Sec. 3.3
 * (set once kappa h is exceeded; the cell then stays SWE).  hsgn_set_mask
 * writes the bytes as given into both step buffers. */
int hsgn_get_mask(hsgn_ctx *c, int patch, uint8_t *m, int on_device);
int hsgn_set_mask(hsgn_ctx *c, int patch, const uint8_t *m, int on_device);

/* Gauges of a scenario at points xy[n][2] (host), the surface-elevation
 * records of the validation cases of Sec. 6.  Each accepted step
 * records eta' = h + b - eta0 (0 in dry cells) interpolated bilinearly
 * between the four nearest cell centres of the finest patch containing the
 * point (patch sets: one record per level-0 step).  Errors: ERANGE. */
int hsgn_set_gauges(hsgn_ctx *c, int scenario, int n, const double *xy);

/* Copy out the gauge records taken since the last read (t[r],
 * eta[r][n]) and forget them.  Host pointers. */
int hsgn_read_gauges(hsgn_ctx *c, int scenario, double *t, double *eta,
                     int max_records, int *n_records);

/* Advance every scenario by n_steps accepted steps.  dt > 0: the same
 * fixed step for every scenario (ECFL if a step's Courant number exceeds
 * cfl_max; that scenario stops at its last good step).  dt < 0: every
 * scenario takes the fixed step set as dt_next by hsgn_set_clock (EINVAL if
 * one is not set).  dt == 0: adaptive step dt_next = dt cfl / Courant with
 * reject and redo above cfl_max; the first step uses
 * cfl / max((|u| + Ce)/dx, (|v| + Ce)/dy).  Patch sets need dt != 0
 * (ENOTSUP) and take n_steps level-0 steps; their whole level-0 step is
 * replayed from a HIP graph when timing is off.  Returns after the device
 * work has completed.  Errors: ECFL, ENONHYP, ENAN, EINVAL, ENOTSUP, EDEVICE. */
int hsgn_advance(hsgn_ctx *c, double dt, int n_steps);

/* Diagnostics of a scenario (patch sets: mass of level 0, counts and cell
 * updates over all levels, clipped mass including refluxing).  The mass is
 * the quantity the conservative update of Sec. 4 keeps up to clipping; the
 * Courant numbers are those of the time-step control of Sec. 4.  Errors:
 * EINVAL. */
int hsgn_diagnostics(hsgn_ctx *c, int scenario, hsgn_diag *d);
/* Clock of a scenario: time t, the next step dt_next (the fixed step, or
 * the adaptive controller's choice dt cfl / Courant of Sec. 4) and the
 * accepted steps.  hsgn_set_clock sets them and clears the scenario's error
 * state (patch sets: given for level 0; level l takes dt_next / 4^l and
 * 4^l steps).  Any output may be NULL.  Errors: EINVAL. */
int hsgn_get_clock(hsgn_ctx *c, int scenario, double *t, double *dt_next,
                   long long *steps);
int hsgn_set_clock(hsgn_ctx *c, int scenario, double t, double dt_next,
                   long long steps);

/* The next three calls are controls of this implementation; no passage of
 * the paper defines them.
 * Tile-height autotuning: for every refinement level, times `trials`
 * step-kernel launches (after one warm-up) for each candidate height in
 * {2, 4, 6, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64} and the height of the
 * library's cost model (the choice with tile_rows <= 0) on the current state, and keeps
 * the fastest.  The state does not advance (the launches write only the
 * spare buffer and the clocks are restored).  rows[nlevels] (may be NULL)
 * receives the chosen heights.  Call after the state is set; drops the
 * captured step graph.  Errors: EINVAL, ENOMEM, EDEVICE. */
int hsgn_autotune(hsgn_ctx *c, int trials, int *rows);

/* Number of marching work items (wavefronts) of one step (a packed item
 * counts once). */
int hsgn_work_items(hsgn_ctx *c, int *n);

/* Kernel timing for measurement: with on = 1, every launch of the step
 * kernel inside hsgn_advance is bracketed by HIP events on the context's
 * stream (patch sets: one launch per level step, launched directly).  hsgn_get_timing returns the summed event time (ms) and the number
 * of launches timed since timing was switched on, then resets both. */
int hsgn_set_timing(hsgn_ctx *c, int on);
int hsgn_get_timing(hsgn_ctx *c, double *step_kernel_ms, long long *launches);

/* Regridding of a patch-set scenario (Sec. 4: Berger-Oliger-Colella
 * adaptive refinement; flagging by the surface jump between neighbouring
 * cells as in the solitary-wave test of Sec. 5).  Call between hsgn_advance
 * calls (all levels are then at the same time).  Level `level` + 1 is
 * rebuilt from flags on level `level`; deeper levels are dropped (regrid
 * them next, level by level).  The rules:
 *   flags    a pair of face neighbours inside a level-l patch, both wet,
 *            whose surface eta' = (h + b) - eta0 differs by more than tol,
 *            flags both cells; then every cell within nbuf cells (max norm,
 *            inside the patch) of a flag;
 *   clusters per level-l patch: a box shrinks to the bounding box of its
 *            flags; with at least `cutoff` of its cells flagged it is
 *            accepted once both sides are <= max_side (else its longer side
 *            is halved, x on ties); otherwise it splits at an empty column or
 *            row of the flag counts nearest the middle (x first, then the
 *            lower index), else at the strongest sign change of their second
 *            difference (sides >= 4; ties: nearest the middle, x, lower
 *            index), else in the middle of the longer side; low half first;
 *   nesting  boxes are clipped to their patch less one cell and refined by
 *            4; new patches follow the patches of their parents and the
 *            order of the clusters;
 *   bottom   a new patch takes the bilinear interpolant of the level-0
 *            bathymetry as set (cell-centred, index coordinates, clamped at
 *            the outer centres); kept patches keep what they were given;
 *            covered coarse cells then take the fine mean;
 *   state    kept cells keep their state (a wet cell whose bathymetry
 *            changed keeps its surface, depth clipped at zero; a dry one
 *            its depth); new cells take the ghost rule's spatial
 *            interpolation from their parent, or a copy where an old
 *            level-(l+1) patch covered them; breaking latches come along;
 *            clocks, clipped mass and unread gauge records carry over.
 * Patch ids change: hsgn_num_patches / hsgn_patch_info list the new patches
 * (every other scenario's patches first in their old order; this scenario's
 * levels <= l, then the new ones).  Tile heights return to the library's
 * choice.  n_new (may be NULL) receives the number of new patches.  Errors:
 * EINVAL (not finalized, bad parameters, bathymetry not set), ENOTSUP (not a
 * patch set, or the context holds a mapped grid, which the rebuilt context
 * would not carry), ENOMEM, EDEVICE; on error the context is unchanged. */
typedef struct hsgn_regrid_params {
    int level;          /* rebuild level + 1 from flags on this level */
    int nbuf;           /* buffer width in level cells (0..64) */
    double tol;         /* surface-jump tolerance (m); negative flags all wet pairs */
    double cutoff;      /* clustering efficiency in (0, 1] */
    int max_side;       /* largest box side in level cells (>= 1) */
} hsgn_regrid_params;
int hsgn_regrid(hsgn_ctx *c, int scenario, const hsgn_regrid_params *r, int *n_new);

/* The patches of a context (the block-structured patches of Sec. 4): their
 * number, and per patch its scenario, refinement level, size, lower-left
 * corner and spacing (any output may be NULL).  Errors: EINVAL. */
int hsgn_num_patches(hsgn_ctx *c, int *n);
int hsgn_patch_info(hsgn_ctx *c, int patch, int *scenario, int *level, int *nx, int *ny,
                    double *x0, double *y0, double *dx, double *dy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one FP64
 * single grid advanced by n_steps fixed steps of dt with no allocation and
 * no context.  It runs the kernels of hsgn_advance (the same bits as a
 * context holding this one grid, FP64, fixed dt).
 *   p          parameters as for hsgn_create; precision must be 0 (FP64,
 *              else ENOTSUP); tile_rows as there
 *   hip_stream borrowed hipStream_t; all work is enqueued on it, and the
 *              call synchronizes it once at the end to read the status
 *   nx, ny     grid size (>= 4); dx, dy spacings; bc[4] as for hsgn_add_grid
 *   b          device pointer, bathymetry [ny][nx] float64 (read only)
 *   q          device pointer, state [7][ny][nx] float64 in conserved
 *              variables (h, hu, hv, hw, h sigma, hp, h p_b), advanced in
 *              place; on ECFL, ENONHYP or ENAN it holds the last good step
 *   steps_done receives the accepted steps (may be NULL)
 * phi_T is derived from b at every call and the breaking latch starts
 * cleared; no gauges, sponge or mapping.  The working memory (spare state
 * buffer, masks, tables: 58 bytes per cell plus a few KB) is a static array
 * of HSGN_STATIC_SCRATCH_MIB MiB per device, reserved when the library is
 * loaded on that device and held until the process ends; grids beyond it
 * return ESCRATCH (about 1.1 M cells: 1024 x 1024 fits).  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be serialized by the caller.
 * Errors: EINVAL, ENOTSUP, ESCRATCH, ECFL, ENONHYP, ENAN, EDEVICE. */
#define HSGN_STATIC_SCRATCH_MIB 64
int hsgn_advance_static(const hsgn_params *p, void *hip_stream, int nx, int ny, double dx,
                        double dy, const int bc[4], const double *b, double *q, double dt,
                        int n_steps, long long *steps_done);

/* Housekeeping, no compute: free a context and its device memory after
 * its stream has drained (NULL: EINVAL); the text of an error code; the message of the last error on a
 * context (valid until its next call). */
int hsgn_destroy(hsgn_ctx *c);
const char *hsgn_strerror(int code);
const char *hsgn_last_error(hsgn_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
