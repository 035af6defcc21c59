/*
 * hsgn_oracle.c -- plain FP64 CPU oracle of the HSGN/SWE time step.
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
 * baseline timing of the benchmark load this file's library.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * Everything here is written for a reader holding the paper:
 *   model      Sec. 3, eq. (HSGN), written in 2D with u = (u, v) and the
 *              scalar sigma = -h div(u) (Sec. 2 notes that the 2D extension
 *              is straightforward);
 *   splitting  Sec. 4: hyperbolic part and algebraic source are split
 *              (Strang by default, Lie selectable);
 *   hyperbolic Sec. 4, eq. (total fluctuation): f-wave decomposition of
 *              F(Q_R) - F(Q_L) plus one-point (Roe-state) quadrature of the
 *              non-conservative and bathymetry integrals, Roe-type averages,
 *              bathymetry sharpness sensor psi, Einfeldt speeds, eigenvectors
 *              of Appendix C; limited second-order corrections (minmod, MC)
 *              and a transverse Riemann solver (wave propagation, Sec. 4);
 *   source     Sec. 4: per-cell linear ODE in (hw, h sigma, hp, h p_b),
 *              integrated with the two-stage L-stable SDIRK(2,2) method;
 *   SWE switch Sec. 3.3 and Sec. 4 (transition function): c^2 = alpha^2 g
 *              H phi_T; cells with phi_T = 0, dry cells and cells latched as
 *              breaking carry no auxiliary variables.
 *   CFL        Sec. 4: global maximum wave speed.
 *   mapped     Sec. 4 (mapped grids, after the cited wave-propagation
 *              treatment of quadrilateral grids): Riemann problems in the
 *              frame of each edge's normal, waves, speeds and fluctuations
 *              scaled by the edge's length ratio, updates divided by the
 *              cell's capacity (area ratio).
 *
 * Readings of points the paper leaves open (c^2 = alpha^2 g H; 2D form;
 * wet/dry states; breaking latch; transverse construction; s = 0 split) are
 * listed in the design notes of the repository and marked at each use below.
 *
 * No blocking, fusion or reordering: every step runs over the whole grid and
 * stores its results in plain arrays before the next step starts.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "hsgn_oracle.h"

/* Working precision.  The oracle is FP64 (real = double).  Built with
 * -DORC_LONG_DOUBLE the same source computes in x87 extended precision
 * (64-bit significand) behind the same FP64 interface: that build measures
 * how far the FP64 evaluation itself is from the exact result of the method
 * on a case (its conditioning); it is never the reference of a parity test. */
#ifdef ORC_LONG_DOUBLE
typedef long double real;
#define sqrt sqrtl
#define fabs fabsl
#define fmin fminl
#define fmax fmaxl
#define floor floorl
#else
typedef double real;
#endif

enum { IH = 0, IHU = 1, IHV = 2, IHW = 3, IHS = 4, IHP = 5, IHPB = 6 };

struct orc_grid {
    orc_params P;
    int nx, ny, sx, sy;         /* sx = nx + 4, sy = ny + 4: two ghost layers */
    real x0, y0, dx, dy;
    int bc[4];
    real *q;                  /* [7][sy][sx] */
    real *b;                  /* [sy][sx] */
    unsigned char *phi;         /* [sy][sx] transition function phi_T */
    unsigned char *brk;         /* [sy][sx] breaking latch */
    /* patch sets: ghosts written by the caller instead of the boundary map,
     * and per-cell flags of edges whose fluxes the caller replaces
     * (bit 0 left, 1 right, 2 bottom, 3 top) */
    int ext_ghosts;
    unsigned char *iface;       /* [sy][sx] */
    /* sponge layer: widths from the domain's x-low, x-high, y-low, y-high
     * sides (0: none), peak rate, and the grid's place in its level's
     * domain (global index of cell (0, 0), domain size in cells) */
    real sp_w[4], sp_rate;
    long long sp_i0, sp_j0, sp_nx, sp_ny;
    /* mapped grid (planar, logically rectangular; NULL on Cartesian grids),
     * [sy][sx] like the cells: kap the cell's capacity (area over dx dy);
     * xn*, xgm the unit normal (towards increasing i) and length ratio
     * (length over dy) of the cell's left edge; yn*, ygm the same for its
     * bottom edge (towards increasing j, length over dx) */
    real *kap, *xnx, *xny, *xgm, *ynx, *yny, *ygm;
    /* radially symmetric solutions (Appendix D): x is the radius */
    int radial;
    real t, dt_next;
    long long nstep, nrej;
    int have_dt;
    real clipped;
    int ngauge;
    real *gxy;
    int nrec, caprec;
    real *rec_t, *rec_eta;
    /* per-step work arrays, allocated on the first step */
    real *w_qs, *w_c2, *w_Flim, *w_Ftr, *w_Glim, *w_Gtr, *w_clip;
    struct edge_s *w_EX, *w_EY;
};

#define CELL(g, i, j) ((size_t)((j) + 2) * (size_t)(g)->sx + (size_t)((i) + 2))
#define PLANE(g) ((size_t)(g)->sx * (size_t)(g)->sy)

/* ------------------------------------------------------------------ */
/* boundary conditions: index map of a ghost cell onto an interior cell */

static int map_index(int i, int n, int lo, int hi, int *flip)
{
    *flip = 0;
    if (i < 0) {
        if (lo == ORC_BC_PERIODIC) return i + n;
        if (lo == ORC_BC_WALL) { *flip = 1; return -1 - i; }
        return 0;
    }
    if (i >= n) {
        if (hi == ORC_BC_PERIODIC) return i - n;
        if (hi == ORC_BC_WALL) { *flip = 1; return 2 * n - 1 - i; }
        return n - 1;
    }
    return i;
}

/* m - 2 (m . n) n: the momentum (hu, hv) mirrored about a wall of unit
 * normal n */
static void reflect(real *hu, real *hv, real nx, real ny)
{
    real a = *hu * nx + *hv * ny;
    *hu = *hu - 2.0 * a * nx;
    *hv = *hv - 2.0 * a * ny;
}

/* fill the two ghost layers of q, b, phi and the latch from the interior */
static void fill_ghosts(orc_grid *g)
{
    size_t np = PLANE(g);
    for (int j = -2; j < g->ny + 2; j++) {
        for (int i = -2; i < g->nx + 2; i++) {
            if (i >= 0 && i < g->nx && j >= 0 && j < g->ny) continue;
            int fx, fy;
            int mi = map_index(i, g->nx, g->bc[0], g->bc[1], &fx);
            int mj = map_index(j, g->ny, g->bc[2], g->bc[3], &fy);
            size_t d = CELL(g, i, j), s = CELL(g, mi, mj);
            for (int m = 0; m < ORC_NV; m++) g->q[m * np + d] = g->q[m * np + s];
            if (g->kap) {
                /* mapped grid: the momentum is mirrored about the wall edge
                 * of the interior cell's row (column) */
                if (fx) {
                    size_t e = CELL(g, i < 0 ? 0 : g->nx, mj);
                    reflect(&g->q[IHU * np + d], &g->q[IHV * np + d], g->xnx[e], g->xny[e]);
                }
                if (fy) {
                    size_t e = CELL(g, mi, j < 0 ? 0 : g->ny);
                    reflect(&g->q[IHU * np + d], &g->q[IHV * np + d], g->ynx[e], g->yny[e]);
                }
            } else {
                if (fx) g->q[IHU * np + d] = -g->q[IHU * np + d];
                if (fy) g->q[IHV * np + d] = -g->q[IHV * np + d];
            }
            g->b[d] = g->b[s];
            g->phi[d] = g->phi[s];
            g->brk[d] = g->brk[s];
        }
    }
}

/* still-water depth H = (eta0 - b)^+ */
static real still_depth(const orc_params *P, real b)
{
    real H = P->eta0 - b;
    return H > 0.0 ? H : 0.0;
}

/* c^2 = alpha^2 g H phi_T, or the fixed c^2 of the run times phi_T; zero in
   SWE cells (phi_T = 0 or breaking) */
static real cell_c2(const orc_grid *g, size_t k)
{
    if (!g->phi[k] || g->brk[k]) return 0.0;
    if (g->P.c2 > 0.0) return g->P.c2;
    return g->P.alpha * g->P.alpha * g->P.g * still_depth(&g->P, g->b[k]);
}

/* ------------------------------------------------------------------ */
/* creation, data in and out                                           */

orc_grid *orc_create(const orc_params *p, int nx, int ny, double x0, double y0,
                     double dx, double dy, const int bc[4])
{
    if (!p || nx < 4 || ny < 4 || !(dx > 0) || !(dy > 0)) return NULL;
    if ((bc[0] == ORC_BC_PERIODIC) != (bc[1] == ORC_BC_PERIODIC)) return NULL;
    if ((bc[2] == ORC_BC_PERIODIC) != (bc[3] == ORC_BC_PERIODIC)) return NULL;
    if (p->nbr_n < 0 || p->nbr_n > 2) return NULL;
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    if (!g) return NULL;
    g->P = *p;
    g->nx = nx; g->ny = ny; g->sx = nx + 4; g->sy = ny + 4;
    g->x0 = x0; g->y0 = y0; g->dx = dx; g->dy = dy;
    memcpy(g->bc, bc, 4 * sizeof(int));
    size_t np = PLANE(g);
    g->q = (real *)calloc(ORC_NV * np, sizeof(real));
    g->b = (real *)calloc(np, sizeof(real));
    g->phi = (unsigned char *)calloc(np, 1);
    g->brk = (unsigned char *)calloc(np, 1);
    g->iface = (unsigned char *)calloc(np, 1);
    if (!g->q || !g->b || !g->phi || !g->brk || !g->iface) { orc_destroy(g); return NULL; }
    return g;
}

void orc_destroy(orc_grid *g)
{
    if (!g) return;
    free(g->q); free(g->b); free(g->phi); free(g->brk); free(g->iface);
    free(g->gxy); free(g->rec_t); free(g->rec_eta);
    free(g->w_qs); free(g->w_c2); free(g->w_Flim); free(g->w_Ftr);
    free(g->w_Glim); free(g->w_Gtr); free(g->w_clip); free(g->w_EX); free(g->w_EY);
    free(g->kap); free(g->xnx); free(g->xny); free(g->xgm);
    free(g->ynx); free(g->yny); free(g->ygm);
    free(g);
}

/* bathymetry and the transition function phi_T (eq. transition function):
 * phi_T = 1 iff the minimum of H over the cells within n cells (max-norm box)
 * exceeds h_star. */
int orc_set_bathymetry(orc_grid *g, const double *b)
{
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++)
            g->b[CELL(g, i, j)] = b[(size_t)j * g->nx + i];
    int n = g->P.nbr_n;
    for (int j = 0; j < g->ny; j++) {
        for (int i = 0; i < g->nx; i++) {
            real hmin = INFINITY;
            for (int dj = -n; dj <= n; dj++) {
                for (int di = -n; di <= n; di++) {
                    int fx, fy;
                    int mi = map_index(i + di, g->nx, g->bc[0], g->bc[1], &fx);
                    int mj = map_index(j + dj, g->ny, g->bc[2], g->bc[3], &fy);
                    real H = still_depth(&g->P, g->b[CELL(g, mi, mj)]);
                    if (H < hmin) hmin = H;
                }
            }
            g->phi[CELL(g, i, j)] = (hmin > g->P.h_star) ? 1 : 0;
            g->brk[CELL(g, i, j)] = 0;
        }
    }
    return ORC_OK;
}

int orc_set_state(orc_grid *g, const double *q)
{
    size_t np = PLANE(g), nn = (size_t)g->nx * g->ny;
    for (int m = 0; m < ORC_NV; m++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++)
                g->q[m * np + CELL(g, i, j)] = q[m * nn + (size_t)j * g->nx + i];
    return ORC_OK;
}

int orc_get_state(const orc_grid *g, double *q)
{
    size_t np = PLANE(g), nn = (size_t)g->nx * g->ny;
    for (int m = 0; m < ORC_NV; m++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++)
                q[m * nn + (size_t)j * g->nx + i] = g->q[m * np + CELL(g, i, j)];
    return ORC_OK;
}

int orc_get_mask(const orc_grid *g, unsigned char *m)
{
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++) {
            size_t k = CELL(g, i, j);
            m[(size_t)j * g->nx + i] = (unsigned char)(g->phi[k] | (g->brk[k] << 1));
        }
    return ORC_OK;
}

int orc_set_mask(orc_grid *g, const unsigned char *m)
{
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++) {
            size_t k = CELL(g, i, j);
            g->phi[k] = m[(size_t)j * g->nx + i] & 1;
            g->brk[k] = (m[(size_t)j * g->nx + i] >> 1) & 1;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* source step (Sec. 4): dY/dt = (1/h) M Y for Y = (hw, h sigma, hp, h p_b),
 * read off the right-hand side of eq. (HSGN):
 *   d(hw)/dt      = p_b
 *   d(h sigma)/dt = -6 p_b + 12 p
 *   d(hp)/dt      = -c^2 sigma
 *   d(h p_b)/dt   = -6 c^2 (w - sigma/2)
 * so M = [[0,0,0,1],[0,0,12,-6],[0,-c^2,0,0],[-6c^2,3c^2,0,0]] acting on
 * (w, sigma, p, p_b), integrated with the two-stage SDIRK(2,2) method with
 * gamma = 1 - 1/sqrt(2): Y1 = Y + gamma tau f(Y1),
 * Y2 = Y + (1-gamma) tau f(Y1) + gamma tau f(Y2), result Y2. */

/* Gaussian elimination with partial pivoting on the n x n system A x = b
 * (row-major A); b is overwritten by x. */
static void solve_lin(int n, real *A, real *b)
{
    for (int k = 0; k < n; k++) {
        int piv = k;
        for (int r = k + 1; r < n; r++)
            if (fabs(A[r * n + k]) > fabs(A[piv * n + k])) piv = r;
        if (piv != k) {
            for (int c = 0; c < n; c++) {
                real t = A[k * n + c]; A[k * n + c] = A[piv * n + c]; A[piv * n + c] = t;
            }
            real t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; r++) {
            real f = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; c++) A[r * n + c] -= f * A[k * n + c];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; k--) {
        real s = b[k];
        for (int c = k + 1; c < n; c++) s -= A[k * n + c] * b[c];
        b[k] = s / A[k * n + k];
    }
}

/* The SDIRK(2,2) step of length tau for dY/dt = J Y / tau with the n x n
 * matrix J = (tau / h) M: stage 1 solves (I - gamma J) Y1 = Y, stage 2
 * solves (I - gamma J) Y2 = Y + (1 - gamma) J Y1; Y2 replaces Y. */
static void sdirk22(int n, const real *J, real *Y)
{
    const real gam = 1.0 - 1.0 / sqrt(2.0);
    real A[16], Y1[4], Y2[4];
    for (int r = 0; r < n; r++)
        for (int c = 0; c < n; c++) A[r * n + c] = (r == c ? 1.0 : 0.0) - gam * J[r * n + c];
    for (int r = 0; r < n; r++) Y1[r] = Y[r];
    solve_lin(n, A, Y1);
    for (int r = 0; r < n; r++) {
        real s = 0.0;
        for (int c = 0; c < n; c++) s += J[r * n + c] * Y1[c];
        Y2[r] = Y[r] + (1.0 - gam) * s;
    }
    for (int r = 0; r < n; r++)
        for (int c = 0; c < n; c++) A[r * n + c] = (r == c ? 1.0 : 0.0) - gam * J[r * n + c];
    solve_lin(n, A, Y2);
    for (int r = 0; r < n; r++) Y[r] = Y2[r];
}

static void source_cell(real *q, real c2, real tau)
{
    const real M[16] = {
        0.0,       0.0,      0.0,  1.0,
        0.0,       0.0,      12.0, -6.0,
        0.0,       -c2,      0.0,  0.0,
        -6.0 * c2, 3.0 * c2, 0.0,  0.0,
    };
    real J[16];
    for (int r = 0; r < 16; r++) J[r] = (tau / q[IH]) * M[r];
    real Y[4] = {q[IHW], q[IHS], q[IHP], q[IHPB]};
    sdirk22(4, J, Y);
    q[IHW] = Y[0]; q[IHS] = Y[1]; q[IHP] = Y[2]; q[IHPB] = Y[3];
}

/* mbHSGN source (Sec. 3, eq. mbHSGN): d(hw)/dt = 3 p / 2 and
 * d(hp)/dt = -2 c^2 w, i.e. dY/dt = (1/h) [[0, 3/2], [-2 c^2, 0]] Y for
 * Y = (hw, hp), by the same SDIRK(2,2). */
static void source_cell_mb(real *q, real c2, real tau)
{
    const real M[4] = {0.0, 1.5, -2.0 * c2, 0.0};
    real J[4];
    for (int r = 0; r < 4; r++) J[r] = (tau / q[IH]) * M[r];
    real Y[2] = {q[IHW], q[IHP]};
    sdirk22(2, J, Y);
    q[IHW] = Y[0]; q[IHP] = Y[1];
}

void orc_source_cell(double *q, double c2, double tau)
{
    real v[7];
    for (int m = 0; m < 7; m++) v[m] = q[m];
    source_cell(v, c2, tau);
    for (int m = 0; m < 7; m++) q[m] = (double)v[m];
}

void orc_source_cell_mb(double *q, double c2, double tau)
{
    real v[7];
    for (int m = 0; m < 7; m++) v[m] = q[m];
    source_cell_mb(v, c2, tau);
    for (int m = 0; m < 7; m++) q[m] = (double)v[m];
}

/* apply the source step of length tau to one cell, or clear the auxiliary
 * variables of a dry or SWE cell (SWE region: c^2 -> 0 with p -> 0) */
/* relaxation rate of the sponge at interior cell (i, j): with d the
 * distance of the cell centre from a sponged side of the domain and w that
 * side's width, s = (w - d) / w inside the band; the largest s over the
 * sides gives sigma = rate s^2 (a reading: the sponge is cited, not
 * described) */
static real sponge_sigma(const orc_grid *g, int i, int j)
{
    const long long I = g->sp_i0 + i, J = g->sp_j0 + j;
    const real d[4] = {((real)I + 0.5) * g->dx, ((real)(g->sp_nx - 1 - I) + 0.5) * g->dx,
                         ((real)J + 0.5) * g->dy, ((real)(g->sp_ny - 1 - J) + 0.5) * g->dy};
    real s = 0.0;
    for (int e = 0; e < 4; e++) {
        const real w = g->sp_w[e];
        if (w > 0.0 && d[e] < w) {
            const real t = (w - d[e]) / w;
            if (t > s) s = t;
        }
    }
    return g->sp_rate * (s * s);
}

static void source_or_clear(orc_grid *g, size_t k, real tau, real *qc)
{
    int wet = qc[IH] > g->P.dry_tol;
    int swe = !g->phi[k] || g->brk[k];
    if (wet && !swe) {
        if (g->P.model == 1) source_cell_mb(qc, cell_c2(g, k), tau);
        else source_cell(qc, cell_c2(g, k), tau);
    } else {
        qc[IHW] = 0.0; qc[IHS] = 0.0; qc[IHP] = 0.0; qc[IHPB] = 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* normal Riemann solver (Sec. 4, eq. total fluctuation; Appendix C)
 *
 * Works in the edge's normal frame: q = (h, h u_n, h u_t, hw, h sigma, hp,
 * h p_b).  The y-direction solve permutes hu and hv before and after. */

typedef struct {
    real uh, vh, wh, sh, ph, pbh;  /* Roe-type averages, normal frame */
    real hh, c2h, ce2;             /* arithmetic means, Ce^2 */
    real smin, smax;               /* Einfeldt speeds */
    int wet;                         /* both cells wet: usable for splitting */
} eig_t;

typedef struct edge_s {
    real Z[7][7];     /* Z[p][m]: f-wave p, component m (normal frame) */
    real s[7];        /* speed of f-wave p */
    real amdq[7], apdq[7];
    int kind;           /* 0 regular, 1 wall (right dry), 2 wall (left dry), 3 dry */
    eig_t e;
} edge_t;

/* bathymetry sharpness sensor psi(b_i, b_{i-1}) of Sec. 4 */
static real sensor(const orc_params *P, real bL, real bR)
{
    real db = bR - bL;
    if (db == 0.0) return 1.0;
    real sum = fabs(bR + bL);
    if (sum == 0.0) return 0.0;
    real xi = 2.0 * fabs(db) / sum;
    if (xi < P->xi0) return 1.0;
    if (xi < P->xi0 + P->xi1) {
        real r = (xi - P->xi0) / P->xi1;
        return -3.0 * r * r + 2.0 * r * r * r + 1.0;
    }
    return 0.0;
}

typedef struct {
    real h, hun, un, ut, w, sg, p, pb, hp;
} side_t;

/* primitive variables of one side; a dry side (h <= dry_tol) keeps its
 * depth, so that a thin film at rest stays in balance, and has zero velocity
 * and auxiliary variables */
static void side_from_q(const orc_params *P, const real *q, side_t *s)
{
    memset(s, 0, sizeof(*s));
    s->h = q[IH] > 0.0 ? q[IH] : 0.0;
    if (q[IH] > P->dry_tol) {
        s->h = q[IH];
        s->hun = q[IHU];
        s->un = q[IHU] / q[IH];
        s->ut = q[IHV] / q[IH];
        s->w = q[IHW] / q[IH];
        s->sg = q[IHS] / q[IH];
        s->p = q[IHP] / q[IH];
        s->pb = q[IHPB] / q[IH];
        s->hp = q[IHP];
    }
}

static int riemann_n(const orc_params *P, const real *qL, const real *qR,
                     real bL, real bR, real c2L, real c2R, edge_t *E)
{
    const real g = P->g;
    memset(E, 0, sizeof(*E));
    int wetL = qL[IH] > P->dry_tol, wetR = qR[IH] > P->dry_tol;
    if (!wetL && !wetR) { E->kind = 3; return ORC_OK; }

    side_t L, R;
    side_from_q(P, qL, &L);
    side_from_q(P, qR, &R);
    real bl = bL, br = bR, cl = c2L, cr = c2R;
    int dryL = 0, dryR = 0;
    /* wet/dry states: a dry neighbour whose bed lies above the wet side's
     * surface acts as a wall (mirror state); otherwise the dry side enters
     * at rest with its own (thin) depth and the dry-front speed bounds the
     * fan. */
    if (wetL && !wetR) {
        if (qL[IH] + bL < bR) {
            E->kind = 1;
            R = L; R.hun = -L.hun; R.un = -L.un;
            br = bl; cr = cl;
        } else {
            dryR = 1;
        }
    } else if (!wetL && wetR) {
        if (qR[IH] + bR < bL) {
            E->kind = 2;
            L = R; L.hun = -R.hun; L.un = -R.un;
            bl = br; cl = cr;
        } else {
            dryL = 1;
        }
    }

    /* Roe-type interface state: arithmetic means of h and c^2, sqrt(h)
     * weighted means of the primitive variables */
    real sqL = sqrt(L.h), sqR = sqrt(R.h);
    real hh = 0.5 * (L.h + R.h);
    real c2h = 0.5 * (cl + cr);
    real uh = (sqR * R.un + sqL * L.un) / (sqL + sqR);
    real vh = (sqR * R.ut + sqL * L.ut) / (sqL + sqR);
    real wh = (sqR * R.w + sqL * L.w) / (sqL + sqR);
    real sh = (sqR * R.sg + sqL * L.sg) / (sqL + sqR);
    real ph = (sqR * R.p + sqL * L.p) / (sqL + sqR);
    real pbh = (sqR * R.pb + sqL * L.pb) / (sqL + sqR);

    real psi = sensor(P, bl, br);
    real db = br - bl;
    real dh = R.h - L.h;
    real deta = (R.h + br) - (L.h + bl);

    /* total fluctuation: flux difference plus one-point quadrature of the
     * non-conservative products and bathymetry terms at the Roe state.
     * The hydrostatic part is written as g h^ (Delta eta), which equals
     * Delta(g h^2 / 2) + g h^ Delta b exactly. */
    real df[7];
    df[0] = R.hun - L.hun;
    df[2] = R.hun * R.ut - L.hun * L.ut;
    df[3] = R.hun * R.w - L.hun * L.w;
    df[4] = R.hun * R.sg - L.hun * L.sg;
    df[6] = (R.hun * R.pb - L.hun * L.pb) - 6.0 * c2h * uh * psi * db;
    if (P->model == 1) {
        /* mbHSGN has no p_b equation: its plane stays zero */
        df[6] = 0.0;
        /* mbHSGN (eq. mbHSGN): momentum bathymetry term (g h + 3/2 psi p) db,
         * hp row d(u h p) + c^2 d(hu) - c^2 u (d eta + psi db) (Sec. 4) */
        df[1] = g * hh * deta + ((R.hun * R.un + R.hp) - (L.hun * L.un + L.hp)) + psi * (1.5 * ph) * db;
        df[5] = ((R.hun * R.p - L.hun * L.p) + c2h * df[0]) - c2h * uh * (deta + psi * db);
    } else {
        df[1] = g * hh * deta + ((R.hun * R.un + R.hp) - (L.hun * L.un + L.hp)) + psi * pbh * db;
        df[5] = (R.hun * (R.p + cr) - L.hun * (L.p + cl)) - c2h * uh * dh;
    }

    /* Einfeldt speeds from the eigenvalue bound u +- sqrt(g h + p + c^2) */
    real ce2 = g * hh + ph + c2h;
    if (!(ce2 > 0.0)) return ORC_ENONHYP;
    real ceh = sqrt(ce2);
    real smin, smax;
    if (dryL) {
        smin = R.un - 2.0 * sqrt(g * R.h);
    } else {
        real a = g * L.h + L.p + cl;
        if (a < 0.0) return ORC_ENONHYP;
        smin = fmin(uh - ceh, L.un - sqrt(a));
    }
    if (dryR) {
        smax = L.un + 2.0 * sqrt(g * L.h);
    } else {
        real a = g * R.h + R.p + cr;
        if (a < 0.0) return ORC_ENONHYP;
        smax = fmax(uh + ceh, R.un + sqrt(a));
    }

    if (cl == 0.0 && cr == 0.0) {
        /* SWE edge (both cells in the SWE region).  The paper leaves this
         * region to a robust SWE solver; here: the HLLE solver in
         * fluctuation form, whose two waves carry the state jump as well as
         * the flux difference (which supplies the entropy dissipation a pure
         * flux-difference split lacks at transonic rarefactions), with the
         * surface elevation in place of h in the state jump so that the
         * ocean at rest stays exactly at rest.  Remaining components travel
         * as contacts at the Roe speed. */
        real dq0 = deta, dq1 = R.hun - L.hun;
        real z1h = smin * ((smax * dq0 - df[0]) / (smax - smin));
        real z1m = smin * ((smax * dq1 - df[1]) / (smax - smin));
        real z7h = smax * ((df[0] - smin * dq0) / (smax - smin));
        real z7m = smax * ((df[1] - smin * dq1) / (smax - smin));
        real S = z1h + z7h;
        real r1[7] = {z1h, z1m, vh * z1h, wh * z1h, sh * z1h, ph * z1h, pbh * z1h};
        real r7[7] = {z7h, z7m, vh * z7h, wh * z7h, sh * z7h, ph * z7h, pbh * z7h};
        for (int m = 0; m < 7; m++) { E->Z[0][m] = r1[m]; E->Z[6][m] = r7[m]; }
        E->Z[1][IHP] = df[5] - ph * S;
        E->Z[2][IHS] = df[4] - sh * S;
        E->Z[3][IHW] = df[3] - wh * S;
        E->Z[4][IHV] = df[2] - vh * S;
        E->Z[5][IHPB] = df[6] - pbh * S;
    } else {
    /* f-wave coefficients: eigenvectors of Appendix C with the Einfeldt
     * speeds in place of u -+ Ce in the two acoustic eigenvectors */
    real b2 = ((c2h + ph) * df[0] - df[5]) / ce2;
    real S = df[0] - b2;
    real T = df[1] - uh * b2;
    real b1 = (smax * S - T) / (smax - smin);
    real b7 = (T - smin * S) / (smax - smin);
    real bs = df[4] - sh * S;
    real bw = df[3] - wh * S;
    real bv = df[2] - vh * S;
    real bpb = df[6] - pbh * S;

    real r1[7] = {1.0, smin, vh, wh, sh, c2h + ph, pbh};
    real r2[7] = {1.0, uh, 0.0, 0.0, 0.0, -g * hh, 0.0};
    real r7[7] = {1.0, smax, vh, wh, sh, c2h + ph, pbh};
    for (int m = 0; m < 7; m++) {
        E->Z[0][m] = b1 * r1[m];
        E->Z[1][m] = b2 * r2[m];
        E->Z[6][m] = b7 * r7[m];
    }
    E->Z[2][IHS] = bs;
    E->Z[3][IHW] = bw;
    E->Z[4][IHV] = bv;
    E->Z[5][IHPB] = bpb;
    }
    E->s[0] = smin;
    for (int p = 1; p < 6; p++) E->s[p] = uh;
    E->s[6] = smax;

    /* fluctuations; a wave of speed exactly zero is split half and half */
    for (int m = 0; m < 7; m++) {
        real am = 0.0, ap = 0.0;
        for (int p = 0; p < 7; p++) {
            if (E->s[p] < 0.0) am += E->Z[p][m];
            else if (E->s[p] > 0.0) ap += E->Z[p][m];
            else { am += 0.5 * E->Z[p][m]; ap += 0.5 * E->Z[p][m]; }
        }
        E->amdq[m] = am;
        E->apdq[m] = ap;
    }
    if (E->kind == 1) for (int m = 0; m < 7; m++) E->apdq[m] = 0.0;
    if (E->kind == 2) for (int m = 0; m < 7; m++) E->amdq[m] = 0.0;

    E->e.uh = uh; E->e.vh = vh; E->e.wh = wh; E->e.sh = sh; E->e.ph = ph; E->e.pbh = pbh;
    E->e.hh = hh; E->e.c2h = c2h; E->e.ce2 = ce2; E->e.smin = smin; E->e.smax = smax;
    E->e.wet = wetL && wetR;
    return ORC_OK;
}

/* swap the hu and hv components (frame change between x and y edges) */
static void swap_uv(real *v)
{
    real t = v[IHU]; v[IHU] = v[IHV]; v[IHV] = t;
}

/* y-edge solve: permute into the normal frame, solve, permute back */
static int riemann_y(const orc_params *P, const real *qL, const real *qR,
                     real bL, real bR, real c2L, real c2R, edge_t *E)
{
    real a[7], c[7];
    memcpy(a, qL, sizeof(a)); memcpy(c, qR, sizeof(c));
    swap_uv(a); swap_uv(c);
    int rc = riemann_n(P, a, c, bL, bR, c2L, c2R, E);
    for (int p = 0; p < 7; p++) swap_uv(E->Z[p]);
    swap_uv(E->amdq); swap_uv(E->apdq);
    return rc;
}

/* mapped grids.  The frame of an edge is its unit normal n and a unit
 * tangent t: t = (-n_y, n_x) at left (x) edges, t = (n_y, -n_x) at bottom
 * (y) edges, so that an axis-aligned grid has the frames of the Cartesian
 * solves (identity at x-edges, the hu/hv swap at y-edges). */
static void to_frame(real *v, real nx, real ny, real tx, real ty)
{
    real hn = v[IHU] * nx + v[IHV] * ny;
    real ht = v[IHU] * tx + v[IHV] * ty;
    v[IHU] = hn; v[IHV] = ht;
}

static void from_frame(real *v, real nx, real ny, real tx, real ty)
{
    real hu = v[IHU] * nx + v[IHV] * tx;
    real hv = v[IHU] * ny + v[IHV] * ty;
    v[IHU] = hu; v[IHV] = hv;
}

/* solve at a mapped edge: rotated data, the normal solve, then waves and
 * fluctuations rotated back to the global frame and, with the speeds,
 * scaled by the edge's length ratio gm.  The Roe state (E->e) stays in the
 * edge's frame, unscaled, for the transverse splits. */
static int riemann_mapped(const orc_params *P, const real *qL, const real *qR,
                          real bL, real bR, real c2L, real c2R, real nx, real ny,
                          real tx, real ty, real gm, edge_t *E)
{
    real a[7], c[7];
    memcpy(a, qL, sizeof(a)); memcpy(c, qR, sizeof(c));
    to_frame(a, nx, ny, tx, ty);
    to_frame(c, nx, ny, tx, ty);
    int rc = riemann_n(P, a, c, bL, bR, c2L, c2R, E);
    for (int p = 0; p < 7; p++) {
        from_frame(E->Z[p], nx, ny, tx, ty);
        for (int m = 0; m < 7; m++) E->Z[p][m] *= gm;
        E->s[p] *= gm;
    }
    from_frame(E->amdq, nx, ny, tx, ty);
    from_frame(E->apdq, nx, ny, tx, ty);
    for (int m = 0; m < 7; m++) { E->amdq[m] *= gm; E->apdq[m] *= gm; }
    return rc;
}

int orc_riemann_x(const orc_params *p, const double *qL, const double *qR,
                  double bL, double bR, double c2L, double c2R,
                  double *waves, double *speeds, double *amdq, double *apdq,
                  int *kind)
{
    edge_t E;
    real a[7], c[7];
    for (int m = 0; m < 7; m++) { a[m] = qL[m]; c[m] = qR[m]; }
    int rc = riemann_n(p, a, c, bL, bR, c2L, c2R, &E);
    for (int q = 0; q < 7; q++) {
        for (int m = 0; m < 7; m++) waves[q * 7 + m] = (double)E.Z[q][m];
        speeds[q] = (double)E.s[q];
    }
    for (int m = 0; m < 7; m++) { amdq[m] = (double)E.amdq[m]; apdq[m] = (double)E.apdq[m]; }
    *kind = E.kind;
    return rc;
}

/* ------------------------------------------------------------------ */
/* transverse splitting: decompose a vector a, given in the normal frame of
 * the splitting edge, on that edge's eigenvectors (same closed form as the
 * normal solve) and return the part moving in direction sgn (B+ or B-) */
static void trans_split(const orc_params *P, const eig_t *e, const real *a,
                        int sgn, real *out)
{
    real g2 = ((e->c2h + e->ph) * a[0] - a[5]) / e->ce2;
    real S = a[0] - g2;
    real T = a[1] - e->uh * g2;
    real g1 = (e->smax * S - T) / (e->smax - e->smin);
    real g7 = (T - e->smin * S) / (e->smax - e->smin);
    real gt = a[2] - e->vh * S;
    real gw = a[3] - e->wh * S;
    real gs = a[4] - e->sh * S;
    real gpb = a[6] - e->pbh * S;
    real s1 = sgn > 0 ? fmax(e->smin, 0.0) : fmin(e->smin, 0.0);
    real sm = sgn > 0 ? fmax(e->uh, 0.0) : fmin(e->uh, 0.0);
    real s7 = sgn > 0 ? fmax(e->smax, 0.0) : fmin(e->smax, 0.0);
    real r1[7] = {1.0, e->smin, e->vh, e->wh, e->sh, e->c2h + e->ph, e->pbh};
    real r2[7] = {1.0, e->uh, 0.0, 0.0, 0.0, -P->g * e->hh, 0.0};
    real r7[7] = {1.0, e->smax, e->vh, e->wh, e->sh, e->c2h + e->ph, e->pbh};
    real mid[7] = {g2 * r2[0], g2 * r2[1], gt, gw, gs, g2 * r2[5], gpb};
    for (int m = 0; m < 7; m++)
        out[m] = s1 * g1 * r1[m] + sm * mid[m] + s7 * g7 * r7[m];
}

/* x-edge fluctuation a (global frame) split by a y-edge (normal frame = y) */
static void split_by_y(const orc_params *P, const eig_t *e, const real *a,
                       int sgn, real *out)
{
    real t[7];
    memcpy(t, a, sizeof(t));
    swap_uv(t);
    trans_split(P, e, t, sgn, out);
    swap_uv(out);
}

/* fluctuation a (global frame) split by a mapped edge with frame (n, t):
 * rotated into the frame, split by the edge's Roe state, rotated back */
static void split_mapped(const orc_params *P, const eig_t *e, const real *a, int sgn,
                         real nx, real ny, real tx, real ty, real *out)
{
    real t[7];
    memcpy(t, a, sizeof(t));
    to_frame(t, nx, ny, tx, ty);
    trans_split(P, e, t, sgn, out);
    from_frame(out, nx, ny, tx, ty);
}

/* ------------------------------------------------------------------ */
/* wave limiter (Sec. 4): minmod or MC applied to each f-wave family */
static real limiter_phi(int lim, real th)
{
    switch (lim) {
    case 1: return fmax(0.0, fmin(1.0, th));
    case 2: return fmax(0.0, fmin(fmin(0.5 * (1.0 + th), 2.0), 2.0 * th));
    case 3: return 1.0;
    default: return 0.0;
    }
}

static real dot7(const real *a, const real *b)
{
    real s = 0.0;
    for (int m = 0; m < 7; m++) s += a[m] * b[m];
    return s;
}

/* limited second-order correction F~ = 1/2 sum_p sgn(s_p)(1 - dt/dx |s_p|) Z~_p
 * of edge E with upwind neighbours El (left/below) and Er (right/above);
 * the Z are in the global frame */
static void correction(int lim, real dtdx, const edge_t *El, const edge_t *E,
                       const edge_t *Er, real *F)
{
    for (int m = 0; m < 7; m++) F[m] = 0.0;
    if (lim == 0 || E->kind != 0) return;
    for (int p = 0; p < 7; p++) {
        real zz = dot7(E->Z[p], E->Z[p]);
        /* a zero wave has no limited part */
        if (zz == 0.0) continue;
        const edge_t *U = E->s[p] > 0.0 ? El : Er;
        real th = dot7(U->Z[p], E->Z[p]) / zz;
        real ph = limiter_phi(lim, th);
        real sg = E->s[p] > 0.0 ? 1.0 : (E->s[p] < 0.0 ? -1.0 : 0.0);
        real c = 0.5 * sg * (1.0 - dtdx * fabs(E->s[p])) * ph;
        for (int m = 0; m < 7; m++) F[m] += c * E->Z[p][m];
    }
}

/* ------------------------------------------------------------------ */
/* radially symmetric solutions (Appendix D).  With x the radius r and u the
 * radial velocity, the 2D system reduces to the 1D one plus the geometric
 * source -(1/r) (hu, hu u, hu w, hu sigma, hu (p + c^2), hu p_b) in the
 * variables (h, hu, hw, h sigma, hp, h p_b); hv stays zero.  The source is
 * integrated by Heun's method (explicit trapezoidal rule, second order) in
 * half steps before and after the step (Strang splitting). */
static void radial_source(const orc_grid *g, size_t k, real r, const real *q, real *s)
{
    for (int m = 0; m < 7; m++) s[m] = 0.0;
    if (!(q[IH] > g->P.dry_tol)) return;
    const real hu = q[IHU];
    s[IH] = -hu / r;
    s[IHU] = -hu * (q[IHU] / q[IH]) / r;
    s[IHW] = -hu * (q[IHW] / q[IH]) / r;
    s[IHS] = -hu * (q[IHS] / q[IH]) / r;
    s[IHP] = -hu * (q[IHP] / q[IH] + cell_c2(g, k)) / r;
    s[IHPB] = -hu * (q[IHPB] / q[IH]) / r;
}

static void radial_half_step(orc_grid *g, real tau)
{
    const size_t np = PLANE(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < g->ny; j++) {
        for (int i = 0; i < g->nx; i++) {
            const size_t k = CELL(g, i, j);
            const real r = g->x0 + ((real)i + 0.5) * g->dx;
            real q[7], k1[7], qs[7], k2[7];
            for (int m = 0; m < 7; m++) q[m] = g->q[m * np + k];
            radial_source(g, k, r, q, k1);
            for (int m = 0; m < 7; m++) qs[m] = q[m] + tau * k1[m];
            radial_source(g, k, r, qs, k2);
            for (int m = 0; m < 7; m++) g->q[m * np + k] = q[m] + 0.5 * tau * (k1[m] + k2[m]);
        }
    }
}

int orc_set_radial(orc_grid *g, int on)
{
    if (on && (g->kap || g->ext_ghosts || g->x0 < 0.0)) return ORC_EINVAL;
    g->radial = on ? 1 : 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* one step                                                             */

static int step_grid(orc_grid *g, real dt, real *courant)
{
    const orc_params *P = &g->P;
    const int nx = g->nx, ny = g->ny;
    const size_t np = PLANE(g);
    const real dtdx = dt / g->dx, dtdy = dt / g->dy;
    const int nxe = nx + 3, nye = nx + 2;          /* edges per row */
    const size_t nex = (size_t)nxe * (ny + 2);     /* x-edges, rows -1..ny */
    const size_t ney = (size_t)nye * (ny + 3);     /* y-edges, rows -1..ny+1 */
    int rc = ORC_OK;

    if (!g->w_qs) {
        g->w_qs = (real *)malloc(ORC_NV * np * sizeof(real));
        g->w_c2 = (real *)malloc(np * sizeof(real));
        g->w_EX = (edge_t *)malloc(nex * sizeof(edge_t));
        g->w_EY = (edge_t *)malloc(ney * sizeof(edge_t));
        g->w_Flim = (real *)malloc(nex * 7 * sizeof(real));
        g->w_Ftr = (real *)malloc(nex * 7 * sizeof(real));
        g->w_Glim = (real *)malloc(ney * 7 * sizeof(real));
        g->w_Gtr = (real *)malloc(ney * 7 * sizeof(real));
        g->w_clip = (real *)malloc((size_t)ny * sizeof(real));
        if (!g->w_qs || !g->w_c2 || !g->w_EX || !g->w_EY || !g->w_Flim || !g->w_Ftr ||
            !g->w_Glim || !g->w_Gtr || !g->w_clip)
            return ORC_ENOMEM;
    }
    real *qs = g->w_qs, *c2 = g->w_c2;
    edge_t *EX = g->w_EX, *EY = g->w_EY;
    real *Flim = g->w_Flim, *Ftr = g->w_Ftr, *Glim = g->w_Glim, *Gtr = g->w_Gtr;
    memset(Flim, 0, nex * 7 * sizeof(real));
    memset(Ftr, 0, nex * 7 * sizeof(real));
    memset(Glim, 0, ney * 7 * sizeof(real));
    memset(Gtr, 0, ney * 7 * sizeof(real));
#define XE(i, j) ((size_t)((j) + 1) * nxe + (size_t)((i) + 1))
#define YE(i, j) ((size_t)((j) + 1) * nye + (size_t)((i) + 1))

    if (g->radial) radial_half_step(g, 0.5 * dt);
    if (!g->ext_ghosts) fill_ghosts(g);

    /* 1. source half step (Strang) on every cell including ghosts; Lie only
     *    clears the auxiliary variables of dry and SWE cells here. */
#pragma omp parallel for schedule(static)
    for (long kk = 0; kk < (long)np; kk++) {
        size_t k = (size_t)kk;
        real qc[7];
        for (int m = 0; m < 7; m++) qc[m] = g->q[m * np + k];
        if (P->splitting) {
            source_or_clear(g, k, 0.5 * dt, qc);
        } else if (qc[IH] <= P->dry_tol || !g->phi[k] || g->brk[k]) {
            qc[IHW] = 0.0; qc[IHS] = 0.0; qc[IHP] = 0.0; qc[IHPB] = 0.0;
        }
        for (int m = 0; m < 7; m++) qs[m * np + k] = qc[m];
        c2[k] = cell_c2(g, k);
    }

    /* 2. normal solves at every x-edge i (between cells i-1 and i) of rows
     *    -1..ny, i = -1..nx+1 */
#pragma omp parallel for schedule(static) reduction(min:rc)
    for (int j = -1; j <= ny; j++) {
        for (int i = -1; i <= nx + 1; i++) {
            size_t kl = CELL(g, i - 1, j), kr = CELL(g, i, j);
            real ql[7], qr[7];
            for (int m = 0; m < 7; m++) { ql[m] = qs[m * np + kl]; qr[m] = qs[m * np + kr]; }
            int r = g->kap ? riemann_mapped(P, ql, qr, g->b[kl], g->b[kr], c2[kl], c2[kr],
                                            g->xnx[kr], g->xny[kr], 0.0 - g->xny[kr], g->xnx[kr],
                                            g->xgm[kr], &EX[XE(i, j)])
                           : riemann_n(P, ql, qr, g->b[kl], g->b[kr], c2[kl], c2[kr], &EX[XE(i, j)]);
            if (r < rc) rc = r;
        }
    }
    /* 3. normal solves at every y-edge j (between cells j-1 and j) of
     *    columns -1..nx, j = -1..ny+1 */
#pragma omp parallel for schedule(static) reduction(min:rc)
    for (int j = -1; j <= ny + 1; j++) {
        for (int i = -1; i <= nx; i++) {
            size_t kl = CELL(g, i, j - 1), kr = CELL(g, i, j);
            real ql[7], qr[7];
            for (int m = 0; m < 7; m++) { ql[m] = qs[m * np + kl]; qr[m] = qs[m * np + kr]; }
            int r = g->kap ? riemann_mapped(P, ql, qr, g->b[kl], g->b[kr], c2[kl], c2[kr],
                                            g->ynx[kr], g->yny[kr], g->yny[kr], 0.0 - g->ynx[kr],
                                            g->ygm[kr], &EY[YE(i, j)])
                           : riemann_y(P, ql, qr, g->b[kl], g->b[kr], c2[kl], c2[kr], &EY[YE(i, j)]);
            if (r < rc) rc = r;
        }
    }
    if (rc != ORC_OK) return rc;

    /* 4. limited corrections at the x-edges i = 0..nx of rows -1..ny and the
     *    y-edges j = 0..ny of columns -1..nx; on a mapped grid the factor
     *    dt/dx is the mean of dt/(kap dx) of the edge's two cells */
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; j++)
        for (int i = 0; i <= nx; i++) {
            real f = g->kap ? 0.5 * (dtdx / g->kap[CELL(g, i - 1, j)] + dtdx / g->kap[CELL(g, i, j)])
                              : dtdx;
            correction(P->limiter, f, &EX[XE(i - 1, j)], &EX[XE(i, j)],
                       &EX[XE(i + 1, j)], &Flim[XE(i, j) * 7]);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; j++)
        for (int i = -1; i <= nx; i++) {
            real f = g->kap ? 0.5 * (dtdy / g->kap[CELL(g, i, j - 1)] + dtdy / g->kap[CELL(g, i, j)])
                              : dtdy;
            correction(P->limiter, f, &EY[YE(i, j - 1)], &EY[YE(i, j)],
                       &EY[YE(i, j + 1)], &Glim[YE(i, j) * 7]);
        }

    /* 5. transverse propagation (wave propagation form, Sec. 4).  Each
     *    x-edge sends A+dQ - F~ into the cell on its right and A-dQ + F~
     *    into the cell on its left (wall and dry edges send nothing).  Each
     *    of these fluctuations is split on its own by the eigenstructure of
     *    the two y-edges of the cell it entered: the part moving up, B+,
     *    by the cell's upper edge, goes into that edge's correction, the
     *    part moving down, B-, by its lower edge, into the lower edge's
     *    correction, each with weight -dt/(2 dx).  That is four splits per
     *    x-edge; y-edges feed the x-edge corrections in the same way with
     *    -dt/(2 dy).  Seen from a y-edge (i, j): up parts of the two
     *    fluctuations entering cell (i, j-1), down parts of the two
     *    entering cell (i, j). */
    if (P->transverse == 2) {
        const real cx = 0.5 * dtdx, cy = 0.5 * dtdy;
#pragma omp parallel for schedule(static)
        for (int j = 0; j <= ny; j++) {
            for (int i = 0; i < nx; i++) {
                const edge_t *ye = &EY[YE(i, j)];
                real *G = &Gtr[YE(i, j) * 7];
                if (!ye->e.wet) continue;
                for (int part = 0; part < 4; part++) {
                    const int row = part < 2 ? j - 1 : j;      /* the cell entered */
                    const int sgn = part < 2 ? 1 : -1;         /* up or down part */
                    const int left = part % 2 == 0;            /* its left x-edge */
                    const edge_t *xe = &EX[XE(left ? i : i + 1, row)];
                    if (xe->kind != 0) continue;
                    const real *F = &Flim[XE(left ? i : i + 1, row) * 7];
                    real a[7], v[7];
                    for (int m = 0; m < 7; m++)
                        a[m] = left ? xe->apdq[m] - F[m] : xe->amdq[m] + F[m];
                    if (g->kap) {
                        /* mapped: split in the edge's frame; the part is
                         * weighted by the edge's length ratio over the
                         * capacity of the cell it entered */
                        const size_t ke = CELL(g, i, j);
                        const real nx_ = g->ynx[ke], ny_ = g->yny[ke];
                        split_mapped(P, &ye->e, a, sgn, nx_, ny_, ny_, 0.0 - nx_, v);
                        const real wgt = g->ygm[ke] / g->kap[CELL(g, i, row)];
                        for (int m = 0; m < 7; m++) G[m] -= cx * (wgt * v[m]);
                    } else {
                        split_by_y(P, &ye->e, a, sgn, v);
                        for (int m = 0; m < 7; m++) G[m] -= cx * v[m];
                    }
                }
            }
        }
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i <= nx; i++) {
                const edge_t *xe = &EX[XE(i, j)];
                real *F = &Ftr[XE(i, j) * 7];
                if (!xe->e.wet) continue;
                for (int part = 0; part < 4; part++) {
                    const int col = part < 2 ? i - 1 : i;      /* the cell entered */
                    const int sgn = part < 2 ? 1 : -1;         /* right or left part */
                    const int low = part % 2 == 0;             /* its lower y-edge */
                    const edge_t *ye = &EY[YE(col, low ? j : j + 1)];
                    if (ye->kind != 0) continue;
                    const real *Gl = &Glim[YE(col, low ? j : j + 1) * 7];
                    real a[7], v[7];
                    for (int m = 0; m < 7; m++)
                        a[m] = low ? ye->apdq[m] - Gl[m] : ye->amdq[m] + Gl[m];
                    if (g->kap) {
                        const size_t ke = CELL(g, i, j);
                        const real nx_ = g->xnx[ke], ny_ = g->xny[ke];
                        split_mapped(P, &xe->e, a, sgn, nx_, ny_, 0.0 - ny_, nx_, v);
                        const real wgt = g->xgm[ke] / g->kap[CELL(g, col, j)];
                        for (int m = 0; m < 7; m++) F[m] -= cy * (wgt * v[m]);
                    } else {
                        trans_split(P, &xe->e, a, sgn, v);
                        for (int m = 0; m < 7; m++) F[m] -= cy * v[m];
                    }
                }
            }
        }
    }

    /* 6. flux-difference update of the interior cells, then
     * 7. the source step (second Strang half, or the whole Lie step), then
     * 8. fix-ups: positivity, dry cells, breaking latch, SWE cells */
#pragma omp parallel for schedule(static) reduction(min:rc)
    for (int j = 0; j < ny; j++) {
        real clip = 0.0;
        for (int i = 0; i < nx; i++) {
            size_t k = CELL(g, i, j);
            size_t xl = XE(i, j), xr = XE(i + 1, j), yb = YE(i, j), yt = YE(i, j + 1);
            /* Q^{n+1} = Q - dt/dx (A+dQ_{i-1/2} + A-dQ_{i+1/2} + F~_{i+1/2} - F~_{i-1/2})
             *             - dt/dy (B+dQ_{j-1/2} + B-dQ_{j+1/2} + G~_{j+1/2} - G~_{j-1/2}),
             * F~ and G~ being the limited corrections plus the transverse
             * terms.  In a patch set, the contributions through an edge
             * shared with a finer patch are left out here; the finer
             * patch's fluxes replace them after its substeps (refluxing). */
            const int fl = g->iface[k];
            /* mapped grids: dt/dx and dt/dy over the cell's capacity */
            const real ddx = g->kap ? dtdx / g->kap[k] : dtdx;
            const real ddy = g->kap ? dtdy / g->kap[k] : dtdy;
            real qc[7];
            for (int m = 0; m < 7; m++) {
                real apl = (fl & 1) ? 0.0 : EX[xl].apdq[m];
                real Fl = (fl & 1) ? 0.0 : Flim[xl * 7 + m] + Ftr[xl * 7 + m];
                real amr = (fl & 2) ? 0.0 : EX[xr].amdq[m];
                real Fr = (fl & 2) ? 0.0 : Flim[xr * 7 + m] + Ftr[xr * 7 + m];
                real bpb = (fl & 4) ? 0.0 : EY[yb].apdq[m];
                real Gb = (fl & 4) ? 0.0 : Glim[yb * 7 + m] + Gtr[yb * 7 + m];
                real bmt = (fl & 8) ? 0.0 : EY[yt].amdq[m];
                real Gt = (fl & 8) ? 0.0 : Glim[yt * 7 + m] + Gtr[yt * 7 + m];
                qc[m] = qs[m * np + k] - ddx * (apl + amr + Fr - Fl) - ddy * (bpb + bmt + Gt - Gb);
            }
            source_or_clear(g, k, P->splitting ? 0.5 * dt : dt, qc);
            /* sponge: every variable relaxed towards the state at rest
             * (h = H, the rest zero) by an implicit Euler step of rate sigma */
            if (g->sp_rate > 0.0) {
                const real sg = sponge_sigma(g, i, j);
                if (sg > 0.0) {
                    const real f = 1.0 / (1.0 + dt * sg);
                    const real H = still_depth(P, g->b[k]);
                    qc[IH] = H + (qc[IH] - H) * f;
                    for (int m = 1; m < 7; m++) qc[m] = qc[m] * f;
                }
            }
            if (qc[IH] < 0.0) {
                clip += -qc[IH] * (g->kap ? g->kap[k] : 1.0) * g->dx * g->dy;
                qc[IH] = 0.0;
            }
            if (qc[IH] <= P->dry_tol) {
                for (int m = 1; m < 7; m++) qc[m] = 0.0;
            } else if (P->kappa > 0.0 && g->phi[k] && !g->brk[k]) {
                real H = still_depth(P, g->b[k]);
                if (qc[IH] + g->b[k] - P->eta0 > P->kappa * H) g->brk[k] = 1;
            }
            if (!g->phi[k] || g->brk[k] || qc[IH] <= P->dry_tol) {
                qc[IHW] = 0.0; qc[IHS] = 0.0; qc[IHP] = 0.0; qc[IHPB] = 0.0;
            }
            for (int m = 0; m < 7; m++) {
                if (!isfinite(qc[m]) && ORC_ENAN < rc) rc = ORC_ENAN;
                g->q[m * np + k] = qc[m];
            }
        }
        g->w_clip[j] = clip;
    }
    for (int j = 0; j < ny; j++) g->clipped += g->w_clip[j];
    if (g->radial) radial_half_step(g, 0.5 * dt);

    /* 9. Courant number from the speeds of the edges of interior cells (on a
     *    mapped grid the scaled speeds over the smaller capacity of the
     *    edge's two cells) */
    {
        real rx = 0.0, ry = 0.0;
        for (int j = 0; j < ny; j++)
            for (int i = 0; i <= nx; i++) {
                real kk = g->kap ? fmin(g->kap[CELL(g, i - 1, j)], g->kap[CELL(g, i, j)]) : 1.0;
                for (int p = 0; p < 7; p++) rx = fmax(rx, fabs(EX[XE(i, j)].s[p]) / kk);
            }
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i < nx; i++) {
                real kk = g->kap ? fmin(g->kap[CELL(g, i, j - 1)], g->kap[CELL(g, i, j)]) : 1.0;
                for (int p = 0; p < 7; p++) ry = fmax(ry, fabs(EY[YE(i, j)].s[p]) / kk);
            }
        *courant = fmax(dt * rx / g->dx, dt * ry / g->dy);
    }
#undef XE
#undef YE
    return rc;
}

int orc_step(orc_grid *g, double dt, double *courant)
{
    real c = 0.0;
    int rc = step_grid(g, dt, &c);
    *courant = (double)c;
    return rc;
}

/* ------------------------------------------------------------------ */
/* time-step control, gauges, diagnostics                               */

static int initial_dt(const orc_grid *g, real *dt0)
{
    const orc_params *P = &g->P;
    size_t np = PLANE(g);
    real mx = 0.0;
    for (int j = 0; j < g->ny; j++) {
        for (int i = 0; i < g->nx; i++) {
            size_t k = CELL(g, i, j);
            real h = g->q[IH * np + k];
            if (h <= P->dry_tol) continue;
            real u = g->q[IHU * np + k] / h, v = g->q[IHV * np + k] / h;
            real p = g->q[IHP * np + k] / h;
            real a = P->g * h + p + cell_c2(g, k);
            if (a < 0.0) return ORC_ENONHYP;
            real ce = sqrt(a);
            mx = fmax(mx, fmax((fabs(u) + ce) / g->dx, (fabs(v) + ce) / g->dy));
        }
    }
    if (!(mx > 0.0)) return ORC_EINVAL;
    *dt0 = P->cfl / mx;
    return ORC_OK;
}

int orc_initial_dt(const orc_grid *g, double *dt0)
{
    real d = 0.0;
    int rc = initial_dt(g, &d);
    *dt0 = (double)d;
    return rc;
}

static real gauge_eta(const orc_grid *g, real gx, real gy)
{
    size_t np = PLANE(g);
    real fx = (gx - g->x0) / g->dx - 0.5;
    real fy = (gy - g->y0) / g->dy - 0.5;
    int i0 = (int)floor(fx), j0 = (int)floor(fy);
    if (i0 < 0) i0 = 0;
    if (i0 > g->nx - 2) i0 = g->nx - 2;
    if (j0 < 0) j0 = 0;
    if (j0 > g->ny - 2) j0 = g->ny - 2;
    real wx = fx - i0, wy = fy - j0;
    wx = fmin(fmax(wx, 0.0), 1.0);
    wy = fmin(fmax(wy, 0.0), 1.0);
    real e[2][2];
    for (int dj = 0; dj < 2; dj++)
        for (int di = 0; di < 2; di++) {
            size_t k = CELL(g, i0 + di, j0 + dj);
            real h = g->q[IH * np + k];
            e[dj][di] = h > g->P.dry_tol ? h + g->b[k] - g->P.eta0 : 0.0;
        }
    return (1.0 - wx) * (1.0 - wy) * e[0][0] + wx * (1.0 - wy) * e[0][1]
         + (1.0 - wx) * wy * e[1][0] + wx * wy * e[1][1];
}

static int record_gauges(orc_grid *g)
{
    if (g->ngauge == 0) return ORC_OK;
    if (g->nrec == g->caprec) {
        int cap = g->caprec ? 2 * g->caprec : 256;
        real *t = (real *)realloc(g->rec_t, (size_t)cap * sizeof(real));
        if (!t) return ORC_ENOMEM;
        g->rec_t = t;
        real *e = (real *)realloc(g->rec_eta, (size_t)cap * g->ngauge * sizeof(real));
        if (!e) return ORC_ENOMEM;
        g->rec_eta = e;
        g->caprec = cap;
    }
    g->rec_t[g->nrec] = g->t;
    for (int k = 0; k < g->ngauge; k++)
        g->rec_eta[(size_t)g->nrec * g->ngauge + k] = gauge_eta(g, g->gxy[2 * k], g->gxy[2 * k + 1]);
    g->nrec++;
    return ORC_OK;
}

int orc_set_gauges(orc_grid *g, int n, const double *xy)
{
    for (int k = 0; k < n; k++) {
        real x = xy[2 * k], y = xy[2 * k + 1];
        if (x < g->x0 || x > g->x0 + g->nx * g->dx || y < g->y0 || y > g->y0 + g->ny * g->dy)
            return ORC_ERANGE;
    }
    free(g->gxy); free(g->rec_t); free(g->rec_eta);
    g->gxy = NULL; g->rec_t = NULL; g->rec_eta = NULL;
    g->nrec = 0; g->caprec = 0; g->ngauge = n;
    if (n > 0) {
        g->gxy = (real *)malloc((size_t)2 * n * sizeof(real));
        if (!g->gxy) return ORC_ENOMEM;
        for (int k = 0; k < 2 * n; k++) g->gxy[k] = xy[k];
    }
    return ORC_OK;
}

int orc_read_gauges(const orc_grid *g, double *t, double *eta, int max_records, int *n_records)
{
    int n = g->nrec < max_records ? g->nrec : max_records;
    for (int r = 0; r < n; r++) {
        t[r] = g->rec_t[r];
        for (int k = 0; k < g->ngauge; k++)
            eta[(size_t)r * g->ngauge + k] = g->rec_eta[(size_t)r * g->ngauge + k];
    }
    *n_records = n;
    return ORC_OK;
}

int orc_advance(orc_grid *g, double dt, int n)
{
    const orc_params *P = &g->P;
    int adaptive = !(dt > 0.0);
    if (adaptive && !g->have_dt) {
        int r = initial_dt(g, &g->dt_next);
        if (r != ORC_OK) return r;
        g->have_dt = 1;
    }
    size_t np = PLANE(g);
    real *save_q = (real *)malloc(ORC_NV * np * sizeof(real));
    unsigned char *save_b = (unsigned char *)malloc(np);
    if (!save_q || !save_b) { free(save_q); free(save_b); return ORC_ENOMEM; }
    int rc = ORC_OK, accepted = 0, rejects_in_row = 0;
    while (accepted < n) {
        real d = adaptive ? g->dt_next : dt;
        real save_clip = g->clipped, cour = 0.0;
        memcpy(save_q, g->q, ORC_NV * np * sizeof(real));
        memcpy(save_b, g->brk, np);
        int r = step_grid(g, d, &cour);
        if (r != ORC_OK || cour > P->cfl_max) {
            memcpy(g->q, save_q, ORC_NV * np * sizeof(real));
            memcpy(g->brk, save_b, np);
            g->clipped = save_clip;
            if (r != ORC_OK) { rc = r; break; }
            if (!adaptive || ++rejects_in_row > 64) { rc = ORC_ECFL; break; }
            g->dt_next = d * P->cfl / cour;
            g->nrej++;
            continue;
        }
        rejects_in_row = 0;
        g->t += d;
        g->nstep++;
        accepted++;
        if (adaptive) {
            if (cour > 0.0) g->dt_next = d * P->cfl / cour;
        } else {
            g->dt_next = d;
        }
        r = record_gauges(g);
        if (r != ORC_OK) { rc = r; break; }
    }
    free(save_q); free(save_b);
    return rc;
}

int orc_get_clock(const orc_grid *g, double *t, double *dt_next, long long *steps,
                  long long *rejected)
{
    *t = g->t; *dt_next = g->have_dt ? g->dt_next : 0.0;
    *steps = g->nstep; *rejected = g->nrej;
    return ORC_OK;
}

int orc_set_clock(orc_grid *g, double t, double dt_next, long long steps)
{
    g->t = t; g->nstep = steps;
    if (dt_next > 0.0) { g->dt_next = dt_next; g->have_dt = 1; }
    else g->have_dt = 0;
    return ORC_OK;
}

double orc_mass(const orc_grid *g)
{
    size_t np = PLANE(g);
    real s = 0.0;
    for (int j = 0; j < g->ny; j++)
        for (int i = 0; i < g->nx; i++)
            s += g->q[IH * np + CELL(g, i, j)] * (g->kap ? g->kap[CELL(g, i, j)] : 1.0);
    return s * g->dx * g->dy;
}

double orc_clipped_mass(const orc_grid *g) { return g->clipped; }

/* ------------------------------------------------------------------ */
/* patch sets (static AMR, Sec. 4 notes the wave-propagation AMR of Berger
 * and LeVeque): the caller owns the ghost frame and the flux registers      */

int orc_framed(orc_grid *g, double **q, double **b, unsigned char **phi,
               unsigned char **brk, unsigned char **iface, int *sx, int *sy)
{
#ifdef ORC_LONG_DOUBLE
    /* the framed arrays are FP64 views: patch sets run in FP64 only */
    (void)q; (void)b; (void)phi; (void)brk; (void)iface; (void)sx; (void)sy;
    return ORC_EINVAL;
#else
    *q = g->q; *b = g->b; *phi = g->phi; *brk = g->brk; *iface = g->iface;
    *sx = g->sx; *sy = g->sy;
    return ORC_OK;
#endif
}

void orc_set_external_ghosts(orc_grid *g, int on) { g->ext_ghosts = on ? 1 : 0; }

int orc_set_sponge(orc_grid *g, const double w[4], double rate, long long i0, long long j0,
                   long long nx_dom, long long ny_dom)
{
    if (!(rate >= 0.0) || !isfinite(rate) || nx_dom < 1 || ny_dom < 1 || i0 < 0 || j0 < 0 ||
        i0 + g->nx > nx_dom || j0 + g->ny > ny_dom)
        return ORC_EINVAL;
    for (int e = 0; e < 4; e++)
        if (!(w[e] >= 0.0) || !isfinite(w[e])) return ORC_EINVAL;
    for (int e = 0; e < 4; e++) g->sp_w[e] = w[e];
    g->sp_rate = rate;
    g->sp_i0 = i0; g->sp_j0 = j0; g->sp_nx = nx_dom; g->sp_ny = ny_dom;
    return ORC_OK;
}

int orc_set_mapping(orc_grid *g, const double *xn, const double *yn)
{
    if (!xn || !yn) return ORC_EINVAL;
    const int W = g->nx + 5;
    const size_t np = PLANE(g);
    real *a[7];
    for (int m = 0; m < 7; m++) {
        a[m] = (real *)malloc(np * sizeof(real));
        if (!a[m]) { for (int k = 0; k <= m; k++) free(a[k]); return ORC_ENOMEM; }
    }
#define NX(i, j) xn[(size_t)((j) + 2) * W + (size_t)((i) + 2)]
#define NY(i, j) yn[(size_t)((j) + 2) * W + (size_t)((i) + 2)]
    int bad = 0;
    for (int j = -2; j < g->ny + 2; j++) {
        for (int i = -2; i < g->nx + 2; i++) {
            const size_t k = CELL(g, i, j);
            /* area from the cross product of the diagonals (counter-clockwise
             * corners (i, j), (i+1, j), (i+1, j+1), (i, j+1)) */
            real area = 0.5 * ((NX(i + 1, j + 1) - NX(i, j)) * (NY(i, j + 1) - NY(i + 1, j))
                               - (NX(i, j + 1) - NX(i + 1, j)) * (NY(i + 1, j + 1) - NY(i, j)));
            /* left edge (i, j) -> (i, j+1), normal towards increasing i */
            real ex = NX(i, j + 1) - NX(i, j), ey = NY(i, j + 1) - NY(i, j);
            real L = sqrt(ex * ex + ey * ey);
            a[0][k] = area / (g->dx * g->dy);
            a[1][k] = ey / L;
            a[2][k] = (0.0 - ex) / L;   /* +0 for an axis-aligned edge */
            a[3][k] = L / g->dy;
            /* bottom edge (i, j) -> (i+1, j), normal towards increasing j */
            real fx = NX(i + 1, j) - NX(i, j), fy = NY(i + 1, j) - NY(i, j);
            real M = sqrt(fx * fx + fy * fy);
            a[4][k] = (0.0 - fy) / M;
            a[5][k] = fx / M;
            a[6][k] = M / g->dx;
            if (!(area > 0.0) || !(L > 0.0) || !(M > 0.0) || !isfinite(area)) bad = 1;
        }
    }
#undef NX
#undef NY
    if (bad) { for (int m = 0; m < 7; m++) free(a[m]); return ORC_EINVAL; }
    free(g->kap); free(g->xnx); free(g->xny); free(g->xgm);
    free(g->ynx); free(g->yny); free(g->ygm);
    g->kap = a[0]; g->xnx = a[1]; g->xny = a[2]; g->xgm = a[3];
    g->ynx = a[4]; g->yny = a[5]; g->ygm = a[6];
    return ORC_OK;
}

int orc_metric(const orc_grid *g, double *out)
{
    if (!g->kap) return ORC_EINVAL;
    const size_t np = PLANE(g);
    const real *pl[7] = {g->kap, g->xnx, g->xny, g->xgm, g->ynx, g->yny, g->ygm};
    for (int m = 0; m < 7; m++)
        for (size_t k = 0; k < np; k++) out[(size_t)m * np + k] = (double)pl[m][k];
    return ORC_OK;
}

/* phi_T of the interior cells from the bathymetry of the frame, ghost cells
 * included (the caller has filled them); clears the breaking latch */
int orc_update_phi_framed(orc_grid *g)
{
    int n = g->P.nbr_n;
    for (int j = 0; j < g->ny; j++) {
        for (int i = 0; i < g->nx; i++) {
            real hmin = INFINITY;
            for (int dj = -n; dj <= n; dj++)
                for (int di = -n; di <= n; di++) {
                    real H = still_depth(&g->P, g->b[CELL(g, i + di, j + dj)]);
                    if (H < hmin) hmin = H;
                }
            g->phi[CELL(g, i, j)] = (hmin > g->P.h_star) ? 1 : 0;
            g->brk[CELL(g, i, j)] = 0;
        }
    }
    return ORC_OK;
}

/* What the last step sent through each boundary edge of the patch, as the
 * flux through the edge minus the flux function of the cell outside it:
 *   left   (x-edge i = 0):   A-dQ + F~ + F~tr
 *   right  (x-edge i = nx): -(A+dQ - F~) + F~tr
 *   bottom (y-edge j = 0):   B-dQ + G~ + G~tr
 *   top    (y-edge j = ny): -(B+dQ - G~) + G~tr
 * K[e][7] with e = j (left), ny + j (right), 2 ny + i (bottom),
 * 2 ny + nx + i (top).  Valid after orc_step. */
int orc_boundary_flux(const orc_grid *g, double *K)
{
    if (!g->w_EX) return ORC_EINVAL;
    const int nx = g->nx, ny = g->ny;
    const int nxe = nx + 3, nye = nx + 2;
#define XE(i, j) ((size_t)((j) + 1) * nxe + (size_t)((i) + 1))
#define YE(i, j) ((size_t)((j) + 1) * nye + (size_t)((i) + 1))
    const edge_t *EX = g->w_EX, *EY = g->w_EY;
    const real *Flim = g->w_Flim, *Ftr = g->w_Ftr, *Glim = g->w_Glim, *Gtr = g->w_Gtr;
    for (int j = 0; j < ny; j++) {
        size_t xl = XE(0, j), xr = XE(nx, j);
        for (int m = 0; m < 7; m++) {
            K[(size_t)j * 7 + m] = (EX[xl].amdq[m] + Flim[xl * 7 + m]) + Ftr[xl * 7 + m];
            K[(size_t)(ny + j) * 7 + m] = -(EX[xr].apdq[m] - Flim[xr * 7 + m]) + Ftr[xr * 7 + m];
        }
    }
    for (int i = 0; i < nx; i++) {
        size_t yb = YE(i, 0), yt = YE(i, ny);
        for (int m = 0; m < 7; m++) {
            K[(size_t)(2 * ny + i) * 7 + m] = (EY[yb].amdq[m] + Glim[yb * 7 + m]) + Gtr[yb * 7 + m];
            K[(size_t)(2 * ny + nx + i) * 7 + m] =
                -(EY[yt].apdq[m] - Glim[yt * 7 + m]) + Gtr[yt * 7 + m];
        }
    }
#undef XE
#undef YE
    return ORC_OK;
}

/* total fluctuation A-dQ + A+dQ of one edge (dir 0: x, 1: y), the
 * non-conservative form of F(Q_R) - F(Q_L) in eq. (total fluctuation) */
int orc_edge_dflux(const orc_params *p, int dir, const double *qL, const double *qR,
                   double bL, double bR, double c2L, double c2R, double *df)
{
    edge_t E;
    real a[7], c[7];
    for (int m = 0; m < 7; m++) { a[m] = qL[m]; c[m] = qR[m]; }
    int rc = dir ? riemann_y(p, a, c, bL, bR, c2L, c2R, &E)
                 : riemann_n(p, a, c, bL, bR, c2L, c2R, &E);
    for (int m = 0; m < 7; m++) df[m] = (double)(E.amdq[m] + E.apdq[m]);
    return rc;
}

/* the same two entry points over n cells / edges (arrays of n 7-vectors) */
void orc_source_cells(int n, double *q, const double *c2, double tau, int model)
{
    for (int k = 0; k < n; k++) {
        if (model == 1) orc_source_cell_mb(q + 7 * (size_t)k, c2[k], tau);
        else orc_source_cell(q + 7 * (size_t)k, c2[k], tau);
    }
}

int orc_edge_dflux_n(const orc_params *p, int dir, int n, const double *qL, const double *qR,
                     const double *bL, const double *bR, const double *c2L, const double *c2R,
                     double *df)
{
    int rc = ORC_OK;
    for (int k = 0; k < n; k++) {
        int r = orc_edge_dflux(p, dir, qL + 7 * (size_t)k, qR + 7 * (size_t)k, bL[k], bR[k],
                               c2L[k], c2R[k], df + 7 * (size_t)k);
        if (r != ORC_OK) rc = r;
    }
    return rc;
}

/* the same for mapped edges: the solve of the mapped step (riemann_mapped)
 * at an edge of unit normal n and length ratio gm, frames as in the step */
int orc_edge_dflux_mapped_n(const orc_params *p, int dir, int n, const double *qL,
                            const double *qR, const double *bL, const double *bR,
                            const double *c2L, const double *c2R, const double *nx,
                            const double *ny, const double *gm, double *df)
{
    int rc = ORC_OK;
    for (int k = 0; k < n; k++) {
        edge_t E;
        real a[7], c[7];
        for (int m = 0; m < 7; m++) { a[m] = qL[7 * (size_t)k + m]; c[m] = qR[7 * (size_t)k + m]; }
        const real tx = dir ? ny[k] : 0.0 - ny[k];
        const real ty = dir ? 0.0 - nx[k] : nx[k];
        int r = riemann_mapped(p, a, c, bL[k], bR[k], c2L[k], c2R[k], nx[k], ny[k], tx, ty,
                               gm[k], &E);
        if (r != ORC_OK) rc = r;
        for (int m = 0; m < 7; m++) df[7 * (size_t)k + m] = (double)(E.amdq[m] + E.apdq[m]);
    }
    return rc;
}

/* limiter function phi(theta) of Sec. 4 (0 first order, 1 minmod, 2 MC,
 * 3 unlimited) */
double orc_limiter_phi(int lim, double theta) { return (double)limiter_phi(lim, theta); }

/* bilinear eta' of the patch at a point (same rule as the gauges) */
double orc_gauge_eta(const orc_grid *g, double x, double y) { return gauge_eta(g, x, y); }
