// hsgn_math.hpp -- per-cell and per-edge arithmetic of the HSGN/SWE step.
//
// Device functions (also compilable as plain host C++) used by the marching
// step kernel: loading a cell, the relaxation source step, the normal
// Riemann solver, the wave limiter and the transverse splitting.
//
//   model        eq. (HSGN), Sec. 3, in 2D with u = (u, v) and the scalar
//                sigma = -h div(u);
//   Riemann      Sec. 4, eq. (total fluctuation): f-wave split of the flux
//                difference plus the Roe-state quadrature of the
//                non-conservative and bathymetry terms, Roe-type averages,
//                sharpness sensor psi, Einfeldt speeds, eigenvectors of
//                Appendix C; in the SWE region (c^2 = 0 on both sides) an
//                HLLE split that carries the surface-elevation jump;
//   limiter      Sec. 4 (minmod, MC) on each wave family;
//   source       Sec. 4, SDIRK(2,2) with gamma = 1 - 1/sqrt(2) on
//                Y = (hw, h sigma, hp, h p_b); the 4x4 stage systems are
//                solved in closed form;
//   SWE switch   Sec. 3.3 / eq. (transition function): c^2 = alpha^2 g H
//                phi_T, zero in breaking cells.
#pragma once

#include <cmath>
#include <cstdint>
#include <type_traits>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define HSGN_HD __host__ __device__ __forceinline__
#define HSGN_UNROLL _Pragma("unroll")
#else
#define HSGN_HD inline
#define HSGN_UNROLL
#endif

namespace hsgn {

enum { IH = 0, IHU = 1, IHV = 2, IHW = 3, IHS = 4, IHP = 5, IHPB = 6 };
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_EXTRAP = 2 };
enum { KIND_REGULAR = 0, KIND_WALL_R = 1, KIND_WALL_L = 2, KIND_DRY = 3 };

// run parameters as the kernels see them
struct StepParams {
    double g;
    double a2g;        // alpha^2 g, or 0 when c^2 is fixed
    double c2f;        // the fixed c^2, or 0: a wet non-SWE cell has
                       // c^2 = a2g H + c2f, one of the two terms zero
    double eta0, h_star, dry_tol, xi0, xi1, kappa;
    int limiter;       // 0 first order, 1 minmod, 2 MC, 3 unlimited
    int transverse;    // 0 none, 2 with corrections
    int splitting;     // 0 Lie, 1 Strang
    int model;         // 0 HSGN, 1 mbHSGN (sigma and p_b stay zero)
};

// one cell after loading and the first source half step
template <class T>
struct Cell {
    T q[7];            // conserved (h, hu, hv, hw, h sigma, hp, h p_b)
    T h;               // max(q[0], 0)
    T sq;              // sqrt(h)
    T ce;              // sqrt(g h + p + c^2) of a wet cell
    T u, v, w, s, p, pb;   // primitives, zero in dry cells
    T b, c2;
    T eta;             // surface for the hydrostatic jump: h + b (FP64) or the
                       // stored deviation eta' (mixed precision, where h + b
                       // would carry the FP32 rounding of a 4000 m depth)
    int wet;           // h > dry_tol
    int hyp;           // g h + p + c^2 >= 0 (always true for a dry cell)
};

// waves of one edge in the global frame.  Families: 0 (speed smin), 1
// (speed uh; nonzero components h, normal momentum, hp), contacts sigma, w,
// tangential momentum, p_b (speed uh), 6 (speed smax).
template <class T>
struct Waves {
    T z0[7], z6[7];
    T zm[3];           // family 1: h, normal momentum, hp
    T bs, bw, bt, bpb; // contact strengths
    T smin, smax, uh;
    int kind;
    // mapped edges only: the edge's frame (unit normal n, tangent t) and
    // length ratio; the waves above are in that frame, the speeds scaled
    T fnx, fny, ftx, fty, gm;
};

// eigenstructure of an edge used to split fluctuations transversally
// (normal frame of that edge)
template <class T>
struct Eig {
    T uh, vh, wh, sh, pbh, ghh, c2p, ce2, inv_ce2, smin, smax, inv_ds;
    int wet;           // both cells wet
    T fnx, fny, ftx, fty, gm;   // mapped edges only: frame and length ratio
};

// larger and smaller of two values, one instruction each on the device for
// float and double.  A NaN operand never decides anything the step keeps (a
// NaN state is reported, not stepped); a zero may come out with either sign.
template <class T>
HSGN_HD T tmax(T a, T b) { return a > b ? a : b; }
template <class T>
HSGN_HD T tmin(T a, T b) { return a < b ? a : b; }
HSGN_HD double tmax(double a, double b) { return fmax(a, b); }
HSGN_HD float tmax(float a, float b) { return fmaxf(a, b); }

// reciprocal used where one denominator serves several quotients, square
// root and quotient.  FP64 on the device: the hardware reciprocal estimate
// refined by two Newton steps (within an ulp or so of 1 / x, in five
// instructions against about ten for the IEEE division), quotients as
// products with it, and the IEEE square root.  FP32 on the device: the bare
// hardware instructions (about 1 ulp); the default FP32 lowering wraps them
// in range scaling for denormal arguments, four or five instructions more
// each, which changes no result for the normal arguments the step passes.
HSGN_HD double recip(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
#else
    return 1.0 / x;
#endif
}
HSGN_HD double tsqrt(double x) { return sqrt(x); }
HSGN_HD double tdiv(double a, double b) { return a * recip(b); }
HSGN_HD float recip(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
HSGN_HD float tsqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
HSGN_HD float tdiv(float a, float b) { return a * recip(b); }

// quotient a / b given inv = 1 / b: a product with the reciprocal
HSGN_HD double quot(double a, double, double inv) { return a * inv; }
HSGN_HD float quot(float a, float, float inv) { return a * inv; }

// sqrt(g h) for the dry-front speed: FP64 evaluates it directly, FP32 reuses
// the cell's sqrt(h)
HSGN_HD double front_root(double g, double h, double, double) { return sqrt(g * h); }
HSGN_HD float front_root(float, float, float sg, float sq) { return sg * sq; }

// reciprocal for the limiter ratios: hardware estimate refined by two
// Newton steps (a few ulp), which is all a ratio fed to a continuous
// limiter function needs
HSGN_HD float frcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// squared wave norms below this are treated as zero waves by the limiter
template <class T> HSGN_HD T tiny_norm();
template <> HSGN_HD double tiny_norm<double>() { return 1e-200; }
template <> HSGN_HD float tiny_norm<float>() { return 1e-30f; }
// finite and of sane magnitude
template <class T> HSGN_HD bool finite_val(T x);
template <> HSGN_HD bool finite_val<double>(double x) { return fabs(x) <= 1e300; }
template <> HSGN_HD bool finite_val<float>(float x) { return fabsf(x) <= 3e38f; }

HSGN_HD double frcp(double x) { return recip(x); }
HSGN_HD double tmin(double a, double b) { return fmin(a, b); }
HSGN_HD float tmin(float a, float b) { return fminf(a, b); }

HSGN_HD int map_index(int i, int n, int lo, int hi, int *flip)
{
    *flip = 0;
    if (i < 0) {
        if (lo == BC_PERIODIC) return i + n;
        if (lo == BC_WALL) { *flip = 1; return -1 - i; }
        return 0;
    }
    if (i >= n) {
        if (hi == BC_PERIODIC) return i - n;
        if (hi == BC_WALL) { *flip = 1; return 2 * n - 1 - i; }
        return n - 1;
    }
    return i;
}

template <class T>
HSGN_HD T still_depth(const StepParams &P, T b)
{
    T H = (T)P.eta0 - b;
    return H > (T)0 ? H : (T)0;
}

// ---------------------------------------------------------------------------
// relaxation source step: (I - k M) X = R solved in closed form, k = gamma
// tau / h, M the 4x4 matrix of the right-hand side of eq. (HSGN) acting on
// (w, sigma, p, p_b):
//   rows  hw: p_b;  h sigma: 12 p - 6 p_b;  hp: -c^2 sigma;
//         h p_b: -6 c^2 w + 3 c^2 sigma
template <class T>
HSGN_HD void stage_solve(T k, T c2, const T R[4], T X[4])
{
    T kc2 = k * c2;
    T a = (T)1 + (T)12 * k * kc2;
    T d = (T)1 + (T)6 * k * kc2;
    T det = a * d + (T)18 * k * kc2;
    T idet = recip(det);
    T r2 = R[1] + (T)12 * k * R[2];
    T r4 = R[3] - (T)6 * kc2 * R[0];
    T x2 = (d * r2 - (T)6 * k * r4) * idet;
    T x4 = (a * r4 + (T)3 * kc2 * r2) * idet;
    X[0] = R[0] + k * x4;
    X[1] = x2;
    X[2] = R[2] - kc2 * x2;
    X[3] = x4;
}

template <class T>
HSGN_HD void source_step(T *q, T c2, T tau)
{
    const T gam = (T)1 - (T)1 / sqrt((T)2);
    T th = quot(tau, q[IH], recip(q[IH]));
    T Y[4] = {q[IHW], q[IHS], q[IHP], q[IHPB]};
    T k = gam * th;
    T Y1[4];
    stage_solve(k, c2, Y, Y1);
    T w = (T)1 - gam;
    T MY[4] = {Y1[3], (T)12 * Y1[2] - (T)6 * Y1[3], -c2 * Y1[1],
               (T)-6 * c2 * Y1[0] + (T)3 * c2 * Y1[1]};
    T R[4];
    HSGN_UNROLL
    for (int m = 0; m < 4; m++) R[m] = Y[m] + w * (th * MY[m]);
    T Y2[4];
    stage_solve(k, c2, R, Y2);
    q[IHW] = Y2[0]; q[IHS] = Y2[1]; q[IHP] = Y2[2]; q[IHPB] = Y2[3];
}

// mbHSGN (eq. mbHSGN): d(hw)/dt = 3 p / 2, d(hp)/dt = -2 c^2 w, by the same
// SDIRK(2,2); a stage (I - k M) X = R has X0 = (R0 + 3/2 k R1) / det,
// X1 = (R1 - 2 c^2 k R0) / det, det = 1 + 3 c^2 k^2
template <class T>
HSGN_HD void stage_solve_mb(T k, T c2, const T R[2], T X[2])
{
    T kc2 = k * c2;
    T idet = recip((T)1 + (T)3 * k * kc2);
    X[0] = (R[0] + (T)1.5 * k * R[1]) * idet;
    X[1] = (R[1] - (T)2 * kc2 * R[0]) * idet;
}

template <class T>
HSGN_HD void source_step_mb(T *q, T c2, T tau)
{
    const T gam = (T)1 - (T)1 / sqrt((T)2);
    T th = quot(tau, q[IH], recip(q[IH]));
    T Y[2] = {q[IHW], q[IHP]};
    T k = gam * th;
    T Y1[2];
    stage_solve_mb(k, c2, Y, Y1);
    T w = (T)1 - gam;
    T MY[2] = {(T)1.5 * Y1[1], (T)-2 * c2 * Y1[0]};
    T R[2];
    HSGN_UNROLL
    for (int m = 0; m < 2; m++) R[m] = Y[m] + w * (th * MY[m]);
    T Y2[2];
    stage_solve_mb(k, c2, R, Y2);
    q[IHW] = Y2[0]; q[IHP] = Y2[1];
}

// source step or clearing of the auxiliary variables (dry or SWE cell)
template <class T>
HSGN_HD void source_or_clear(const StepParams &P, T *q, T c2, int swe, T tau)
{
    if (q[IH] > (T)P.dry_tol && !swe) {
        if (P.model == 1) source_step_mb(q, c2, tau);
        else source_step(q, c2, tau);
    } else {
        q[IHW] = (T)0; q[IHS] = (T)0; q[IHP] = (T)0; q[IHPB] = (T)0;
    }
}

// fill the derived fields of a cell from its conserved variables
template <class T>
HSGN_HD void derive(const StepParams &P, Cell<T> &c)
{
    c.h = c.q[IH] > (T)0 ? c.q[IH] : (T)0;
    c.sq = tsqrt(c.h);
    c.wet = c.q[IH] > (T)P.dry_tol;
    c.hyp = 1;
    c.ce = (T)0;
    if (c.wet) {
        T h = c.q[IH];
        T ih = recip(h);
        c.u = c.q[IHU] * ih; c.v = c.q[IHV] * ih;
        c.w = c.q[IHW] * ih; c.s = c.q[IHS] * ih;
        c.p = c.q[IHP] * ih; c.pb = c.q[IHPB] * ih;
        T a = (T)P.g * c.h + c.p + c.c2;
        c.hyp = a >= (T)0;
        c.ce = tsqrt(a > (T)0 ? a : (T)0);
    } else {
        c.u = c.v = c.w = c.s = c.p = c.pb = (T)0;
    }
}

// bathymetry sharpness sensor psi of Sec. 4
template <class T>
HSGN_HD T sensor(const StepParams &P, T bL, T bR)
{
    // every case is formed and the result selected, without branches (a
    // zero sum's infinite or undefined ratio is dropped by the selects):
    // 1 for a flat bottom or xi < xi0, the ramp 1 - 3 r^2 + 2 r^3 for
    // xi0 <= xi < xi0 + xi1, else 0 (also for bR + bL = 0 with bR != bL)
    const T db = bR - bL;
    const T sum = fabs(bR + bL);
    const T num = (T)2 * fabs(db);
    const T xi = tdiv(num, sum);
    const T r = tdiv(xi - (T)P.xi0, (T)P.xi1);
    const T ramp = (T)-3 * r * r + (T)2 * r * r * r + (T)1;
    const T tail = xi < (T)(P.xi0 + P.xi1) ? ramp : (T)0;
    const T psi = xi < (T)P.xi0 ? (T)1 : tail;
    return db == (T)0 ? (T)1 : (sum == (T)0 ? (T)0 : psi);
}

// ---------------------------------------------------------------------------
// normal Riemann solve.  DIR = 0: x-edge (normal momentum hu), DIR = 1:
// y-edge (normal momentum hv).  Returns false if the edge is not hyperbolic.
// one side of an edge in the edge's normal frame: what the normal solve
// needs of a cell (a dry cell keeps its thin depth and has zero velocity and
// auxiliaries)
template <class T>
struct Side {
    T h, sq, ce, hun, un, ut, w, s, p, pb, hp, b, c2, eta;
    int wet, hyp;
};

template <int DIR, class T>
HSGN_HD void side_of(const Cell<T> &c, Side<T> &sd)
{
    const int IN = DIR == 0 ? IHU : IHV;
    sd.h = c.h;
    sd.sq = c.sq;
    sd.ce = c.ce;
    sd.wet = c.wet;
    sd.hyp = c.hyp;
    sd.b = c.b;
    sd.c2 = c.c2;
    sd.eta = c.eta;
    // the primitives of a dry cell are zero already (derive); its momentum
    // and hp count as zero too
    sd.un = DIR == 0 ? c.u : c.v;
    sd.ut = DIR == 0 ? c.v : c.u;
    sd.w = c.w; sd.s = c.s; sd.p = c.p; sd.pb = c.pb;
    sd.hun = c.wet ? c.q[IN] : (T)0;
    sd.hp = c.wet ? c.q[IHP] : (T)0;
}

// WET: compiled for edges whose two sides are wet (no dry, wall or
// dry-front case); the caller takes it only when that holds for every edge
// of the wavefront it uses (the results are those of the general solve)
template <int DIR, bool WET = false, class T>
HSGN_HD bool riemann(const StepParams &P, const Side<T> &sL, const Side<T> &sR,
                     Waves<T> &W, Eig<T> &E)
{
    const int IN = DIR == 0 ? IHU : IHV;   // normal momentum component
    const int IT = DIR == 0 ? IHV : IHU;   // tangential momentum component
    const T g = (T)P.g;
    E.wet = WET ? 1 : (sL.wet && sR.wet);
    if (!WET && !sL.wet && !sR.wet) {
        // both sides dry: no waves
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) { W.z0[m] = (T)0; W.z6[m] = (T)0; }
        W.zm[0] = W.zm[1] = W.zm[2] = (T)0;
        W.bs = W.bw = W.bt = W.bpb = (T)0;
        W.smin = W.smax = W.uh = (T)0;
        W.kind = KIND_DRY;
        E.uh = E.vh = E.wh = E.sh = E.pbh = E.ghh = E.c2p = (T)0;
        E.ce2 = (T)1; E.inv_ce2 = (T)1; E.smin = (T)-1; E.smax = (T)1; E.inv_ds = (T)0.5;
        return true;
    }
    // Every other path assigns every output; a non-hyperbolic edge clears
    // `ok` and runs on (its outputs are then meaningless: the step reports
    // the edge), so that no output has to be set before a branch.
    bool ok = true;
    W.kind = KIND_REGULAR;
    Side<T> L = sL, R = sR;
    int dryL = 0, dryR = 0;
    if (!WET && sL.wet && !sR.wet) {
        if (sL.h + sL.b < sR.b) {
            W.kind = KIND_WALL_R;
            R = L; R.hun = -L.hun; R.un = -L.un;
        } else {
            dryR = 1;
        }
    } else if (!WET && !sL.wet && sR.wet) {
        if (sR.h + sR.b < sL.b) {
            W.kind = KIND_WALL_L;
            L = R; L.hun = -R.hun; L.un = -R.un;
        } else {
            dryL = 1;
        }
    }

    T sqL = L.sq, sqR = R.sq;
    T den = sqL + sqR;
    T iden = recip(den);
    T hh = (T)0.5 * (L.h + R.h);
    T c2h = (T)0.5 * (L.c2 + R.c2);
    T uh = (sqR * R.un + sqL * L.un) * iden;
    T vh = (sqR * R.ut + sqL * L.ut) * iden;
    T wh = (sqR * R.w + sqL * L.w) * iden;
    T sh = (sqR * R.s + sqL * L.s) * iden;
    T ph = (sqR * R.p + sqL * L.p) * iden;
    T pbh = (sqR * R.pb + sqL * L.pb) * iden;

    T psi = sensor(P, L.b, R.b);
    T db = R.b - L.b;
    T dh = R.h - L.h;
    T deta = R.eta - L.eta;

    T df[7];
    df[0] = R.hun - L.hun;
    df[2] = R.hun * R.ut - L.hun * L.ut;
    df[3] = R.hun * R.w - L.hun * L.w;
    df[4] = R.hun * R.s - L.hun * L.s;
    const bool mb = P.model == 1;
    if (mb) {
        // mbHSGN: (g h + 3/2 psi p) db in the momentum, and the hp row
        // d(u h p) + c^2 d(hu) - c^2 u (d eta + psi db); no p_b equation
        df[1] = g * hh * deta + ((R.hun * R.un + R.hp) - (L.hun * L.un + L.hp)) + psi * ((T)1.5 * ph) * db;
        df[5] = ((R.hun * R.p - L.hun * L.p) + c2h * df[0]) - c2h * uh * (deta + psi * db);
        df[6] = (T)0;
    } else {
        df[1] = g * hh * deta + ((R.hun * R.un + R.hp) - (L.hun * L.un + L.hp)) + psi * pbh * db;
        df[5] = (R.hun * (R.p + R.c2) - L.hun * (L.p + L.c2)) - c2h * uh * dh;
        df[6] = (R.hun * R.pb - L.hun * L.pb) - (T)6 * c2h * uh * psi * db;
    }

    T ce2 = g * hh + ph + c2h;
    ok = ce2 > (T)0;
    T ceh = tsqrt(ce2);
    T ice2 = recip(ce2);
    T sg = tsqrt(g);
    T smin, smax;
    if (dryL) {
        smin = R.un - (T)2 * front_root(g, R.h, sg, R.sq);
    } else {
        ok = ok && L.hyp;
        smin = tmin(uh - ceh, L.un - L.ce);
    }
    if (dryR) {
        smax = L.un + (T)2 * front_root(g, L.h, sg, L.sq);
    } else {
        ok = ok && R.hyp;
        smax = tmax(uh + ceh, R.un + R.ce);
    }
    T ids = recip(smax - smin);

    // normal-frame waves, then scattered into the global frame.  An edge
    // with c^2 = 0 on both sides takes the SWE waves; FP32 solves never do:
    // in mixed precision every edge with c^2 = 0 on a side is solved again
    // in FP64, whose results replace the FP32 ones
    T n0[7], n6[7];
    if (!std::is_same<T, float>::value && L.c2 == (T)0 && R.c2 == (T)0) {
        // SWE edge: HLLE waves carrying the surface-elevation jump
        T dq0 = deta, dq1 = R.hun - L.hun;
        T z1h = smin * ((smax * dq0 - df[0]) * ids);
        T z1m = smin * ((smax * dq1 - df[1]) * ids);
        T z7h = smax * ((df[0] - smin * dq0) * ids);
        T z7m = smax * ((df[1] - smin * dq1) * ids);
        T S = z1h + z7h;
        n0[0] = z1h; n0[1] = z1m; n0[2] = vh * z1h; n0[3] = wh * z1h;
        n0[4] = sh * z1h; n0[5] = ph * z1h; n0[6] = pbh * z1h;
        n6[0] = z7h; n6[1] = z7m; n6[2] = vh * z7h; n6[3] = wh * z7h;
        n6[4] = sh * z7h; n6[5] = ph * z7h; n6[6] = pbh * z7h;
        W.zm[0] = (T)0; W.zm[1] = (T)0; W.zm[2] = df[5] - ph * S;
        W.bs = df[4] - sh * S;
        W.bw = df[3] - wh * S;
        W.bt = df[2] - vh * S;
        W.bpb = df[6] - pbh * S;
    } else {
        // strength of the wave at speed u_hat: ((c2 + p)_hat df1 - df6) / Ce^2.
        // In FP32 the two terms (each about c^2 hu, 1e7 in deep water) are
        // expanded so that the c^2 parts cancel exactly:
        //   c2_hat (hu_R - hu_L) - (hu_R c2_R - hu_L c2_L)
        //     = -(c2_R - c2_L) (hu_R + hu_L) / 2,
        // leaving no difference of large numbers.  FP64 keeps the plain form.
        T num;
        if constexpr (sizeof(T) == 4) {
            if (mb)   // the c^2 d(hu) parts cancel exactly
                num = ph * df[0] - (R.hun * R.p - L.hun * L.p) + c2h * uh * (deta + psi * db);
            else
                num = ph * df[0] - (R.hun * R.p - L.hun * L.p)
                    - (T)0.5 * (R.c2 - L.c2) * (R.hun + L.hun) + c2h * uh * dh;
        } else {
            num = (c2h + ph) * df[0] - df[5];
        }
        T b2 = num * ice2;
        T S = df[0] - b2;
        T Tm = df[1] - uh * b2;
        T b1 = (smax * S - Tm) * ids;
        T b7 = (Tm - smin * S) * ids;
        n0[0] = b1; n0[1] = b1 * smin; n0[2] = b1 * vh; n0[3] = b1 * wh;
        n0[4] = b1 * sh; n0[5] = b1 * (c2h + ph); n0[6] = b1 * pbh;
        n6[0] = b7; n6[1] = b7 * smax; n6[2] = b7 * vh; n6[3] = b7 * wh;
        n6[4] = b7 * sh; n6[5] = b7 * (c2h + ph); n6[6] = b7 * pbh;
        W.zm[0] = b2; W.zm[1] = b2 * uh; W.zm[2] = b2 * (-g * hh);
        W.bs = df[4] - sh * S;
        W.bw = df[3] - wh * S;
        W.bt = df[2] - vh * S;
        W.bpb = df[6] - pbh * S;
    }
    W.z0[IH] = n0[0]; W.z0[IN] = n0[1]; W.z0[IT] = n0[2];
    W.z6[IH] = n6[0]; W.z6[IN] = n6[1]; W.z6[IT] = n6[2];
    HSGN_UNROLL
    for (int m = 3; m < 7; m++) { W.z0[m] = n0[m]; W.z6[m] = n6[m]; }
    W.smin = smin; W.smax = smax; W.uh = uh;

    E.uh = uh; E.vh = vh; E.wh = wh; E.sh = sh; E.pbh = pbh;
    E.ghh = g * hh; E.c2p = c2h + ph; E.ce2 = ce2; E.inv_ce2 = ice2; E.smin = smin; E.smax = smax;
    E.inv_ds = ids;
    return ok;
}

// precision conversion of solver results
template <class D, class T>
HSGN_HD void convert(const Waves<T> &a, Waves<D> &o)
{
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) { o.z0[m] = (D)a.z0[m]; o.z6[m] = (D)a.z6[m]; }
    o.zm[0] = (D)a.zm[0]; o.zm[1] = (D)a.zm[1]; o.zm[2] = (D)a.zm[2];
    o.bs = (D)a.bs; o.bw = (D)a.bw; o.bt = (D)a.bt; o.bpb = (D)a.bpb;
    o.smin = (D)a.smin; o.smax = (D)a.smax; o.uh = (D)a.uh;
    o.kind = a.kind;
}

template <class D, class T>
HSGN_HD void convert(const Eig<T> &a, Eig<D> &o)
{
    o.uh = (D)a.uh; o.vh = (D)a.vh; o.wh = (D)a.wh; o.sh = (D)a.sh; o.pbh = (D)a.pbh;
    o.ghh = (D)a.ghh; o.c2p = (D)a.c2p; o.ce2 = (D)a.ce2; o.inv_ce2 = (D)a.inv_ce2;
    o.smin = (D)a.smin; o.smax = (D)a.smax; o.inv_ds = (D)a.inv_ds;
    o.wet = a.wet;
}

template <class D, class T>
HSGN_HD void convert(const Side<T> &a, Side<D> &o)
{
    o.h = (D)a.h; o.sq = (D)a.sq; o.ce = (D)a.ce; o.hun = (D)a.hun; o.un = (D)a.un;
    o.ut = (D)a.ut; o.w = (D)a.w; o.s = (D)a.s; o.p = (D)a.p; o.pb = (D)a.pb;
    o.hp = (D)a.hp; o.b = (D)a.b; o.c2 = (D)a.c2; o.eta = (D)a.eta;
    o.wet = a.wet; o.hyp = a.hyp;
}

// full 7-vector of family f of the waves (global frame); DIR selects where
// the normal-momentum component of family 1 and the tangential contact sit
template <int DIR, class T>
HSGN_HD void wave_vec(const Waves<T> &W, int f, T *z)
{
    if constexpr (DIR == 2) {
        // mapped edge: the frame wave rotated back to the global frame and
        // scaled by the edge's length ratio
        wave_vec<0>(W, f, z);
        const T hu = z[IHU] * W.fnx + z[IHV] * W.ftx;
        const T hv = z[IHU] * W.fny + z[IHV] * W.fty;
        z[IHU] = hu; z[IHV] = hv;
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) z[m] = z[m] * W.gm;
    } else {
        const int IN = DIR == 0 ? IHU : IHV;
        const int IT = DIR == 0 ? IHV : IHU;
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) z[m] = (T)0;
        switch (f) {
        case 0: for (int m = 0; m < 7; m++) z[m] = W.z0[m]; break;
        case 1: z[IH] = W.zm[0]; z[IN] = W.zm[1]; z[IHP] = W.zm[2]; break;
        case 2: z[IHS] = W.bs; break;
        case 3: z[IHW] = W.bw; break;
        case 4: z[IT] = W.bt; break;
        case 5: z[IHPB] = W.bpb; break;
        default: for (int m = 0; m < 7; m++) z[m] = W.z6[m]; break;
        }
    }
}

template <class T>
HSGN_HD T wave_speed(const Waves<T> &W, int f)
{
    return f == 0 ? W.smin : (f == 6 ? W.smax : W.uh);
}

// dot products of the 7 families of two edges (same direction)
template <int DIR, class T>
HSGN_HD void family_dots(const Waves<T> &A, const Waves<T> &B, T *d)
{
    HSGN_UNROLL
    for (int f = 0; f < 7; f++) {
        T za[7], zb[7];
        wave_vec<DIR>(A, f, za);
        wave_vec<DIR>(B, f, zb);
        T s = (T)0;
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) s += za[m] * zb[m];
        d[f] = s;
    }
}

// the limiters of the wave-propagation correction as one branch-free form
//   phi(th) = max(e, min(a th, b, c th + d))
// with per-launch coefficients: minmod max(0, min(1, th)) (a, b, c, d, e) =
// (1, 1, 0, 1, 0); MC max(0, min((1 + th) / 2, 2, 2 th)) = (2, 2, 1/2, 1/2, 0)
// (th / 2 + 1 / 2 rounds once, as (1 + th) / 2 does); Lax-Wendroff 1 =
// (0, 0, 0, 0, 1); none 0 = all zero
template <class T>
struct Limiter {
    T a, b, c, d, e;
};

template <class T>
HSGN_HD Limiter<T> limiter_of(int lim)
{
    if (lim == 1) return {(T)1, (T)1, (T)0, (T)1, (T)0};
    if (lim == 2) return {(T)2, (T)2, (T)0.5, (T)0.5, (T)0};
    if (lim == 3) return {(T)0, (T)0, (T)0, (T)0, (T)1};
    return {(T)0, (T)0, (T)0, (T)0, (T)0};
}

template <class T>
HSGN_HD T limiter_phi(const Limiter<T> &L, T th)
{
    return tmax(L.e, tmin(tmin(L.a * th, L.b), L.c * th + L.d));
}

// sum_f c_f Z_f over the seven families of an edge (DIR 0 or 1: the
// families' nonzero components only; the two acoustic waves are full
// vectors, the u-speed family has h, normal momentum and hp components, the
// four contact waves one component each)
template <int DIR, class T>
HSGN_HD void family_sum(const Waves<T> &W, const T *c, T *out)
{
    if constexpr (DIR == 2) {
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) out[m] = (T)0;
        HSGN_UNROLL
        for (int f = 0; f < 7; f++) {
            T z[7];
            wave_vec<DIR>(W, f, z);
            HSGN_UNROLL
            for (int m = 0; m < 7; m++) out[m] += c[f] * z[m];
        }
    } else {
        const int IN = DIR == 0 ? IHU : IHV;
        const int IT = DIR == 0 ? IHV : IHU;
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) out[m] = c[0] * W.z0[m] + c[6] * W.z6[m];
        out[IH] += c[1] * W.zm[0];
        out[IN] += c[1] * W.zm[1];
        out[IHP] += c[1] * W.zm[2];
        out[IHS] += c[2] * W.bs;
        out[IHW] += c[3] * W.bw;
        out[IT] += c[4] * W.bt;
        out[IHPB] += c[5] * W.bpb;
    }
}

// limited second-order correction of an edge from its own waves and the dot
// products with the left (dl) and right (dr) neighbouring edges; an edge
// that is not regular (wall, dry) has none
template <int DIR, class T>
HSGN_HD void correction(const Limiter<T> &lim, T dtdx, const Waves<T> &W, const T *dl,
                        const T *dr, T *F)
{
    const bool on = W.kind == KIND_REGULAR;
    T self[7], c[7];
    family_dots<DIR>(W, W, self);
    HSGN_UNROLL
    for (int f = 0; f < 7; f++) {
        T zz = self[f];
        T s = wave_speed(W, f);
        // waves this small contribute nothing at the working precision;
        // skipping them also keeps the reciprocal of zz finite
        const bool live = on && zz > tiny_norm<T>();
        const T th = live ? quot(s > (T)0 ? dl[f] : dr[f], zz, frcp(zz)) : (T)0;
        const T ph = live ? limiter_phi(lim, th) : (T)0;
        T sg = s > (T)0 ? (T)1 : (s < (T)0 ? (T)-1 : (T)0);
        c[f] = (T)0.5 * sg * ((T)1 - dtdx * fabs(s)) * ph;
    }
    family_sum<DIR>(W, c, F);
}

// left- and right-going fluctuations; a wave of speed exactly zero is split
// half and half
template <int DIR, class T>
HSGN_HD void fluctuations(const Waves<T> &W, T *am, T *ap)
{
    T wm[7], wp[7];
    HSGN_UNROLL
    for (int f = 0; f < 7; f++) {
        T s = wave_speed(W, f);
        wm[f] = s < (T)0 ? (T)1 : (s > (T)0 ? (T)0 : (T)0.5);
        wp[f] = s > (T)0 ? (T)1 : (s < (T)0 ? (T)0 : (T)0.5);
    }
    family_sum<DIR>(W, wm, am);
    family_sum<DIR>(W, wp, ap);
    const T km = W.kind == KIND_WALL_L ? (T)0 : (T)1;
    const T kp = W.kind == KIND_WALL_R ? (T)0 : (T)1;
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) { am[m] *= km; ap[m] *= kp; }
}

// transverse split of a global-frame vector a by the eigenstructure E of an
// edge of direction DIR: returns the part moving with sign sgn
template <int DIR, class T>
HSGN_HD void trans_split(const Eig<T> &E, const T *a, int sgn, T *out)
{
    if constexpr (DIR == 2) {
        // mapped edge: a rotated into the edge's frame, split there, the
        // parts rotated back
        T t[7];
        HSGN_UNROLL
        for (int m = 0; m < 7; m++) t[m] = a[m];
        t[IHU] = a[IHU] * E.fnx + a[IHV] * E.fny;
        t[IHV] = a[IHU] * E.ftx + a[IHV] * E.fty;
        trans_split<0>(E, t, sgn, out);
        const T hu = out[IHU] * E.fnx + out[IHV] * E.ftx;
        const T hv = out[IHU] * E.fny + out[IHV] * E.fty;
        out[IHU] = hu; out[IHV] = hv;
        return;
    }
    const int IN = DIR == 0 ? IHU : IHV;
    const int IT = DIR == 0 ? IHV : IHU;
    T an[7] = {a[IH], a[IN], a[IT], a[IHW], a[IHS], a[IHP], a[IHPB]};
    T g2 = (E.c2p * an[0] - an[5]) * E.inv_ce2;
    T S = an[0] - g2;
    T Tm = an[1] - E.uh * g2;
    T g1 = (E.smax * S - Tm) * E.inv_ds;
    T g7 = (Tm - E.smin * S) * E.inv_ds;
    T gt = an[2] - E.vh * S;
    T gw = an[3] - E.wh * S;
    T gs = an[4] - E.sh * S;
    T gpb = an[6] - E.pbh * S;
    T s1 = sgn > 0 ? tmax(E.smin, (T)0) : tmin(E.smin, (T)0);
    T sm = sgn > 0 ? tmax(E.uh, (T)0) : tmin(E.uh, (T)0);
    T s7 = sgn > 0 ? tmax(E.smax, (T)0) : tmin(E.smax, (T)0);
    T r1[7] = {(T)1, E.smin, E.vh, E.wh, E.sh, E.c2p, E.pbh};
    T r7[7] = {(T)1, E.smax, E.vh, E.wh, E.sh, E.c2p, E.pbh};
    T mid[7] = {g2, g2 * E.uh, gt, gw, gs, g2 * (-E.ghh), gpb};
    T on[7];
    HSGN_UNROLL
    for (int m = 0; m < 7; m++) on[m] = s1 * g1 * r1[m] + sm * mid[m] + s7 * g7 * r7[m];
    out[IH] = on[0]; out[IN] = on[1]; out[IT] = on[2];
    HSGN_UNROLL
    for (int m = 3; m < 7; m++) out[m] = on[m];
}

}  // namespace hsgn
