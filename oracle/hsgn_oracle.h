/*
 * hsgn_oracle.h -- interface of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the
 * smoke check and the CPU-baseline timing can compare the GPU library
 * against a slow, obviously correct statement of the method.  No product
 * code links, loads or calls it.  It shares no source with the GPU path.
 *
 * What it computes: one explicit finite-volume step of the hyperbolic
 * Serre-Green-Naghdi system (HSGN, Sec. 3, eq. HSGN) on a 2D Cartesian
 * grid, in the wave-propagation form of Sec. 4 (f-wave normal Riemann
 * solver with Roe-type interface state and Einfeldt speeds, limited
 * second-order corrections, transverse Riemann solver), with the SDIRK(2,2)
 * relaxation source step (Sec. 4) applied by Strang or Lie splitting and the
 * cell-wise switch to the shallow water equations through the transition
 * function phi_T and c^2 = alpha^2 g H phi_T (Sec. 3.3, eq. transition
 * function).
 *
 * State layout at this interface: q[7][ny][nx], row-major, conserved
 * variables in the order of Appendix C: h, hu, hv, hw, h*sigma, hp, h*p_b.
 *
 * Precision: FP64.  Compiled with -DORC_LONG_DOUBLE the same source computes
 * in x87 extended precision behind this same FP64 interface (orc_framed is
 * then refused); that build measures the FP64 oracle's own rounding error.
 */
#ifndef HSGN_ORACLE_H
#define HSGN_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NV 7

/* status codes (same meaning as the GPU library's, defined independently) */
#define ORC_OK          0
#define ORC_EINVAL     -1
#define ORC_ENOMEM     -2
#define ORC_ECFL       -3
#define ORC_ENONHYP    -4
#define ORC_ENAN       -5
#define ORC_ERANGE     -6

/* boundary conditions, one per side: x-low, x-high, y-low, y-high */
#define ORC_BC_PERIODIC 0
#define ORC_BC_WALL     1
#define ORC_BC_EXTRAP   2

typedef struct orc_params {
    double g;           /* gravity */
    double alpha;       /* relaxation parameter alpha = c / sqrt(g H) */
    double eta0;        /* sea level at rest */
    double h_star;      /* transition depth for phi_T */
    double dry_tol;     /* h <= dry_tol is dry */
    double xi0, xi1;    /* bathymetry sharpness sensor parameters */
    double cfl;         /* desired Courant number (adaptive dt) */
    double cfl_max;     /* largest accepted Courant number */
    double kappa;       /* breaking latch: eta - eta0 > kappa H (<= 0: off) */
    int nbr_n;          /* neighbourhood half-width n of phi_T */
    int limiter;        /* 0 first order, 1 minmod, 2 MC, 3 unlimited */
    int transverse;     /* 0 none, 2 transverse incl. corrections */
    int splitting;      /* 0 Lie, 1 Strang */
    int model;          /* 0 HSGN (eq. HSGN), 1 mbHSGN (eq. mbHSGN: sigma and
                           p_b stay zero) */
    double c2;          /* > 0: a fixed relaxation parameter c^2 in place of
                           alpha^2 g H (the steady states of Sec. 5 fix c^2);
                           still zero in SWE cells */
} orc_params;

typedef struct orc_grid orc_grid;

orc_grid *orc_create(const orc_params *p, int nx, int ny, double x0, double y0,
                     double dx, double dy, const int bc[4]);
void orc_destroy(orc_grid *g);

/* b[ny][nx]; computes H = (eta0 - b)^+ and phi_T */
int orc_set_bathymetry(orc_grid *g, const double *b);
int orc_set_state(orc_grid *g, const double *q);
int orc_get_state(const orc_grid *g, double *q);
/* mask byte per cell: bit0 = phi_T, bit1 = breaking latch */
int orc_get_mask(const orc_grid *g, unsigned char *m);
int orc_set_mask(orc_grid *g, const unsigned char *m);

/* One step attempt of size dt from the current state.  Always replaces the
 * state with Q^{n+1}; *courant receives the Courant number of the step. */
int orc_step(orc_grid *g, double dt, double *courant);

/* Driver: n accepted steps.  dt > 0: fixed step, returns ORC_ECFL (state
 * left at the last good step) if the Courant number exceeds cfl_max.
 * dt <= 0: adaptive step with reject and redo. */
int orc_advance(orc_grid *g, double dt, int n);
int orc_initial_dt(const orc_grid *g, double *dt0);
int orc_get_clock(const orc_grid *g, double *t, double *dt_next,
                  long long *steps, long long *rejected);
int orc_set_clock(orc_grid *g, double t, double dt_next, long long steps);

int orc_set_gauges(orc_grid *g, int n, const double *xy);
int orc_read_gauges(const orc_grid *g, double *t, double *eta, int max_records,
                    int *n_records);
double orc_mass(const orc_grid *g);
double orc_clipped_mass(const orc_grid *g);

/* Unit-level entry points used by the pin tests. */
/* x-direction f-wave solve of one edge.  waves[p*7+m] = component m of
 * f-wave p, speeds[p], fluctuations amdq/apdq, kind (0 regular, 1 wall with
 * the right cell dry, 2 wall with the left cell dry, 3 both dry). */
int orc_riemann_x(const orc_params *p, const double *qL, const double *qR,
                  double bL, double bR, double c2L, double c2R,
                  double *waves, double *speeds, double *amdq, double *apdq,
                  int *kind);
/* SDIRK(2,2) source step of length tau on one cell (in place): HSGN
 * (4x4 system in hw, h sigma, hp, h p_b) and mbHSGN (2x2 in hw, hp). */
void orc_source_cell(double *q, double c2, double tau);
void orc_source_cell_mb(double *q, double c2, double tau);

/* Patch sets.  orc_framed exposes the grid's framed arrays ([7][sy][sx]
 * state, [sy][sx] bathymetry, phi_T, latch and interface flags; sx = nx+4,
 * sy = ny+4, interior cell (i, j) at (j+2) sx + i+2).  With external ghosts
 * on, orc_step uses the ghost cells as the caller left them.  Interface
 * flag bits (0 left, 1 right, 2 bottom, 3 top) drop the contributions of
 * that edge from the cell's update. */
int orc_framed(orc_grid *g, double **q, double **b, unsigned char **phi,
               unsigned char **brk, unsigned char **iface, int *sx, int *sy);
void orc_set_external_ghosts(orc_grid *g, int on);
/* sponge layer (the relaxation sponge of the Tohoku case, Sec. 6.4, cited
 * there without a description): widths w[4] in metres from the x-low,
 * x-high, y-low, y-high sides of the domain (0: none) and peak rate (1/s).
 * The grid's cell (0, 0) is cell (i0, j0) of a domain of nx_dom x ny_dom
 * cells of its spacing (a single grid: 0, 0, nx, ny). */
int orc_set_sponge(orc_grid *g, const double w[4], double rate, long long i0, long long j0,
                   long long nx_dom, long long ny_dom);
int orc_update_phi_framed(orc_grid *g);
/* mapped grid (Sec. 4, mapped grids): node coordinates xn, yn of a planar
 * logically rectangular grid, [ny + 5][nx + 5], node (i, j) for i = -2..nx+2
 * and j = -2..ny+2 at [j + 2][i + 2] (the two ghost layers included); cell
 * (i, j) has corners (i, j), (i+1, j), (i+1, j+1), (i, j+1) counter-clockwise.
 * The grid's dx and dy become the computational spacings: capacities are
 * areas over dx dy, edge length ratios lengths over dy (left edges) and dx
 * (bottom edges).  Momenta are in the physical frame; walls mirror them about
 * the wall edge (on a patch-set grid the caller fills the ghost cells, walls
 * included).  Refused (ORC_EINVAL) for a cell of non-positive area or an edge
 * of zero length. */
int orc_set_mapping(orc_grid *g, const double *xn, const double *yn);
/* the metric planes of a mapped grid copied to out[7][sy][sx]: capacity;
 * unit normal (x, y) and length ratio of the cell's left edge; the same for
 * its bottom edge.  ORC_EINVAL on a Cartesian grid. */
int orc_metric(const orc_grid *g, double *out);
/* radially symmetric solutions (Appendix D): the grid's x is the radius
 * (x0 >= 0), u the radial velocity, and every step adds the geometric
 * source -(1/r) (hu, hu u, 0, hu w, hu sigma, hu (p + c^2), hu p_b) by
 * Heun's method in half steps before and after it.  Refused on mapped and
 * patch-set grids and for x0 < 0. */
int orc_set_radial(orc_grid *g, int on);
/* boundary-edge fluxes of the last step relative to the outside cell,
 * K[2 ny + 2 nx][7] (left rows, right rows, bottom columns, top columns) */
int orc_boundary_flux(const orc_grid *g, double *K);
/* orc_source_cell(_mb) and orc_edge_dflux over n cells / edges, 7-vectors
 * in a row (model 1: mbHSGN) */
void orc_source_cells(int n, double *q, const double *c2, double tau, int model);
int orc_edge_dflux_n(const orc_params *p, int dir, int n, const double *qL, const double *qR,
                     const double *bL, const double *bR, const double *c2L, const double *c2R,
                     double *df);
/* total fluctuation of n mapped edges in the global frame (dir 0: left
 * edges, tangent (-n_y, n_x); 1: bottom edges, tangent (n_y, -n_x)): the
 * normal solve of the states rotated into the frame of the unit normal
 * (nx, ny), its fluctuations rotated back and scaled by the length ratio gm */
int orc_edge_dflux_mapped_n(const orc_params *p, int dir, int n, const double *qL,
                            const double *qR, const double *bL, const double *bR,
                            const double *c2L, const double *c2R, const double *nx,
                            const double *ny, const double *gm, double *df);
/* limiter function phi(theta): lim 0 first order, 1 minmod, 2 MC, 3 none */
double orc_limiter_phi(int lim, double theta);
/* eta' at a point by the gauge rule (bilinear over the 4 nearest centres) */
double orc_gauge_eta(const orc_grid *g, double x, double y);
/* A-dQ + A+dQ of one edge, dir 0 = x, 1 = y */
int orc_edge_dflux(const orc_params *p, int dir, const double *qL, const double *qR,
                   double bL, double bR, double c2L, double c2R, double *df);

#ifdef __cplusplus
}
#endif
#endif
