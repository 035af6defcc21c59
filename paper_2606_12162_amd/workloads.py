"""Seeded synthetic inputs for the HSGN/SWE time step.

This module holds input generation only (bathymetry, initial states, gauge
positions and run parameters).  It contains none of the time step's
arithmetic; both the GPU library's callers and the oracle-based tests take
their inputs from here.

Closed-form initial data used here:
  * SGN solitary wave (Appendix B).  The printed non-hydrostatic pressure is
    garbled; ``sgn_soliton`` uses p = (h^2/3)(u_x^2 + (c0 - u) u_xx), the SGN
    pressure of a wave travelling at speed c0, written out in closed form.
    On a flat bottom the HSGN auxiliary variables follow from the SGN
    constraints: sigma = -h u_x = 2 w and p_b = 3 p / 2.
  * Linear well-prepared pressure of a surface perturbation at rest over a
    flat bottom (Sec. 3.2): p^ = -(g H^2/3) |k|^2 eta^ / (1 + H^2 |k|^2 / 3)
    on a periodic grid, with w = sigma = 0 and p_b = 3 p / 2.

Variable order of every state array: h, hu, hv, hw, h*sigma, hp, h*p_b, laid
out as q[7][ny][nx] (float64, C order).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

G = 9.81
BC_PERIODIC, BC_WALL, BC_EXTRAP = 0, 1, 2


@dataclasses.dataclass
class Params:
    """Run parameters of the method (Sec. 4 defaults: Courant 0.9-1,
    xi0 = 0.01, xi1 = 0.05, alpha = 3, neighbourhood n = 1)."""
    g: float = G
    alpha: float = 3.0
    eta0: float = 0.0
    h_star: float = 0.0
    dry_tol: float = 1e-3
    xi0: float = 0.01
    xi1: float = 0.05
    cfl: float = 0.9
    cfl_max: float = 1.0
    kappa: float = 0.0
    nbr_n: int = 1
    limiter: int = 2          # 0 first order, 1 minmod, 2 MC, 3 unlimited
    transverse: int = 2       # 0 none, 2 with corrections
    splitting: int = 1        # 0 Lie, 1 Strang
    model: int = 0            # 0 HSGN, 1 mbHSGN
    c2: float = 0.0           # > 0: fixed c^2 (m^2/s^2) instead of alpha^2 g H


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    x0: float
    y0: float
    dx: float
    dy: float
    bc: tuple          # (x-low, x-high, y-low, y-high)


@dataclasses.dataclass
class Workload:
    name: str
    params: Params
    grid: Grid
    b: np.ndarray              # [ny, nx]
    q: np.ndarray              # [7, ny, nx]
    gauges: np.ndarray         # [n, 2]
    steps: int
    dt: float                  # > 0 fixed step, <= 0 adaptive
    amplitude: float           # wave amplitude used to normalise gauge errors


def cell_centres(grid: Grid):
    x = grid.x0 + (np.arange(grid.nx) + 0.5) * grid.dx
    y = grid.y0 + (np.arange(grid.ny) + 0.5) * grid.dy
    return np.meshgrid(x, y)   # X[j, i], Y[j, i]


def fp32_representable(a: np.ndarray) -> np.ndarray:
    """Round to the nearest float32 value (kept as float64), so that a
    bathymetry is stored identically in single and double precision."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# closed-form initial data

def sgn_soliton(x, t, a, H, x0, g=G, direction=1.0):
    """SGN solitary wave of Appendix B: returns h, u, w, p on points x.

    l = sqrt((H^3/a + H^2) 4/3), c0 = sqrt(g (H + a)), xi = x - c0 t - x0,
    h = H + a sech^2(xi/l), u = c0 (1 - H/h), w = -h u_x / 2, and the SGN
    pressure of a travelling wave p = (h^2/3)(u_x^2 + (c0 - u) u_xx)."""
    ell = math.sqrt((H ** 3 / a + H ** 2) * 4.0 / 3.0)
    c0 = direction * math.sqrt(g * (H + a))
    z = (np.asarray(x, dtype=np.float64) - c0 * t - x0) / ell
    sech = 1.0 / np.cosh(z)
    th = np.tanh(z)
    s2 = sech * sech
    h = H + a * s2
    hx = -2.0 * a * s2 * th / ell
    hxx = 2.0 * a * s2 * (2.0 * th * th - s2) / ell ** 2
    u = c0 * (1.0 - H / h)
    ux = c0 * H * hx / h ** 2
    uxx = c0 * H * (hxx / h ** 2 - 2.0 * hx * hx / h ** 3)
    w = -0.5 * h * ux
    p = (h * h / 3.0) * (ux * ux + (c0 - u) * uxx)
    return h, u, w, p


def sgn_soliton_state(x, t, a, H, x0, g=G, direction=1.0):
    """HSGN conserved variables (h, hu, hw, h sigma, hp, h p_b) of the SGN
    soliton on a flat bottom: sigma = 2 w, p_b = 3 p / 2."""
    h, u, w, p = sgn_soliton(x, t, a, H, x0, g, direction)
    return h, h * u, h * w, h * 2.0 * w, h * p, h * 1.5 * p


def linear_prepared_pressure(eta, H, dx, dy, g=G):
    """Non-hydrostatic pressure p of a flat-bottom surface perturbation at
    rest, from the linearised SGN relation on a periodic grid."""
    ny, nx = eta.shape
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dy)
    KX, KY = np.meshgrid(kx, ky)
    k2 = KX * KX + KY * KY
    ph = -(g * H * H / 3.0) * k2 * np.fft.fft2(eta) / (1.0 + H * H * k2 / 3.0)
    return np.real(np.fft.ifft2(ph))


# ---------------------------------------------------------------------------
# the five workloads

def gaussian_hump(n=128, dx=0.1, amplitude=0.05, width=1.0, H=1.0, alpha=3.0,
                  steps=200):
    """Flat bottom of depth H, periodic, Gaussian surface hump at rest with
    well-prepared auxiliary variables; MC, Strang, CFL 0.9 adaptive."""
    grid = Grid(n, n, 0.0, 0.0, dx, dx, (BC_PERIODIC,) * 4)
    X, Y = cell_centres(grid)
    L = n * dx
    r2 = (X - 0.5 * L) ** 2 + (Y - 0.5 * L) ** 2
    eta = amplitude * np.exp(-r2 / width ** 2)
    b = np.full((n, n), -H)
    h = H + eta
    p = linear_prepared_pressure(eta, H, dx, dx)
    q = np.zeros((7, n, n))
    q[0] = h
    q[5] = h * p
    q[6] = 1.5 * h * p
    s = np.linspace(0.1 * L, 0.9 * L, 8)
    gauges = np.stack([s, s], axis=1)
    params = Params(alpha=alpha, h_star=0.0, kappa=0.0)
    return Workload("gaussian_hump_%dx%d_fp64" % (n, n), params, grid, b, q,
                    gauges, steps, 0.0, amplitude)


# --------------------------------------------------------------------------
# radially symmetric hump (Sec. 5, radially symmetric tests): h = H + A
# exp(-r^2 / sigma^2) at rest over a flat bottom, r measured from the
# origin; the quarter domain [0, L]^2 has walls on its left and bottom sides
# and extrapolation on the others.  Auxiliary variables start at zero (the
# same data for the 2D runs and for the radial 1D reference).

RADIAL = dict(H=100.0, A=5.0, sigma=100.0, alpha=3.0)


def _radial_state(R, H, A, sigma):
    q = np.zeros((7,) + R.shape)
    q[0] = H + A * np.exp(-(R / sigma) ** 2)
    return q


def _radial_dt(dx, t_end, H, A, alpha, cfl=0.9):
    """a fixed step no larger than cfl dx / max Ce that divides t_end"""
    ce = math.sqrt(G * (H + A) + alpha * alpha * G * H)
    n = int(math.ceil(t_end / (cfl * dx / ce)))
    return t_end / n, n


def radial_hump(n=48, dx=50.0, t_end=12.0, **kw):
    """the 2D quarter domain on one grid"""
    c = dict(RADIAL, **kw)
    grid = Grid(n, n, 0.0, 0.0, dx, dx, (BC_WALL, BC_EXTRAP, BC_WALL, BC_EXTRAP))
    X, Y = cell_centres(grid)
    q = _radial_state(np.sqrt(X ** 2 + Y ** 2), c["H"], c["A"], c["sigma"])
    dt, steps = _radial_dt(dx, t_end, c["H"], c["A"], c["alpha"])
    params = Params(alpha=c["alpha"], h_star=0.0, kappa=0.0)
    return Workload("radial_hump_%dx%d" % (n, n), params, grid, np.full((n, n), -c["H"]), q,
                    np.zeros((0, 2)), steps, dt, c["A"])


def radial_hump_amr(n0=48, dx0=50.0, t_end=6.0, **kw):
    """the hump at the centre c of the whole domain [0, n0 dx0]^2
    (extrapolation on every side) as a three-level patch set (ratios 4, 4)
    with the same physical layout at every dx0 that divides 50 m: level 0
    one n0 x n0 grid; level 1 the square [c - 400 m, c + 400 m)^2; level 2
    the square [c - 100 m, c + 100 m)^2.  The radius is measured from c."""
    c = dict(RADIAL, **kw)
    bc = (BC_EXTRAP,) * 4
    ctr = 0.5 * n0 * dx0
    specs = [(0, n0, n0, 0.0, 0.0)]
    for lev, half in ((1, 400.0), (2, 100.0)):
        side = int(round(2.0 * half / (dx0 / RATIO ** lev)))
        specs.append((lev, side, side, ctr - half, ctr - half))
    patches = []
    for lev, nx, ny, x0, y0 in specs:
        d = dx0 / RATIO ** lev
        g = Grid(nx, ny, x0, y0, d, d, bc)
        X, Y = cell_centres(g)
        R = np.sqrt((X - ctr) ** 2 + (Y - ctr) ** 2)
        patches.append(PatchSpec(lev, nx, ny, x0, y0, np.full((ny, nx), -c["H"]),
                                 _radial_state(R, c["H"], c["A"], c["sigma"])))
    dt, steps = _radial_dt(dx0, t_end, c["H"], c["A"], c["alpha"])
    params = Params(alpha=c["alpha"], h_star=0.0, kappa=0.0)
    return AmrWorkload("radial_hump_amr_%d" % n0, params, dx0, dx0, bc, patches,
                       np.zeros((0, 2)), steps, dt, c["A"])


def radial_strip(nr=7200, dr=0.5, t_end=12.0, **kw):
    """the radial 1D reference problem: x is the radius, a strip of 4 rows
    (periodic across), a wall at r = 0 and extrapolation at the far end"""
    c = dict(RADIAL, **kw)
    grid = Grid(nr, 4, 0.0, 0.0, dr, dr, (BC_WALL, BC_EXTRAP, BC_PERIODIC, BC_PERIODIC))
    X, _ = cell_centres(grid)
    q = _radial_state(X, c["H"], c["A"], c["sigma"])
    dt, steps = _radial_dt(dr, t_end, c["H"], c["A"], c["alpha"])
    params = Params(alpha=c["alpha"], h_star=0.0, kappa=0.0)
    return Workload("radial_strip_%d" % nr, params, grid, np.full((4, nr), -c["H"]), q,
                    np.zeros((0, 2)), steps, dt, c["A"])


BEACH_GAUGE_X = (10.0, 15.0, 20.0, 25.0, 30.0, 35.0, 38.4, 40.0, 42.0, 44.0,
                 45.0, 46.0, 47.0, 48.0, 48.5, 49.0)


def beach_soliton(n=1024, dx=0.05, a=0.2, H=1.0, x0=15.0, alpha=3.0,
                  steps=2000):
    """Plane beach: depth H for x <= 0.75 L, then the bottom rises linearly to
    +0.2 at x = L; SGN soliton of amplitude a heading shoreward; walls on all
    sides; SWE for H < 0.05 (n = 1 neighbourhood) or breaking; 16 gauges."""
    grid = Grid(n, n, 0.0, 0.0, dx, dx, (BC_WALL,) * 4)
    X, Y = cell_centres(grid)
    L = n * dx
    xs = 0.75 * L
    b = np.where(X <= xs, -H, -H + (0.2 + H) * (X - xs) / (L - xs))
    b = fp32_representable(b)
    q = np.zeros((7, n, n))
    h0, hu0, hw0, hs0, hp0, hpb0 = sgn_soliton_state(X, 0.0, a, H, x0)
    flat = b == -H
    h = np.where(flat, h0, np.maximum(-b, 0.0))
    q[0] = h
    q[1] = np.where(flat, hu0, 0.0)
    q[3] = np.where(flat, hw0, 0.0)
    q[4] = np.where(flat, hs0, 0.0)
    q[5] = np.where(flat, hp0, 0.0)
    q[6] = np.where(flat, hpb0, 0.0)
    gauges = np.array([[gx, 0.5 * L] for gx in BEACH_GAUGE_X])
    params = Params(alpha=alpha, h_star=0.05, kappa=0.8, dry_tol=1e-3)
    return Workload("beach_soliton_%dx%d_fp64" % (n, n), params, grid, b, q,
                    gauges, steps, 0.0, a)


def _ocean_profile(d, L):
    """Depth profile across the shelf, breakpoints as fractions of L:
    -4000 m abyssal plain, slope to -150 m, shelf, linear rise to +30 m."""
    f = d / L
    f1, f2, f3 = 600.0 / 1024.0, 700.0 / 1024.0, 950.0 / 1024.0
    b = np.where(f < f1, -4000.0,
                 np.where(f < f2, -4000.0 + (f - f1) / (f2 - f1) * 3850.0,
                          np.where(f < f3, -150.0,
                                   -150.0 + (f - f3) / (1.0 - f3) * 180.0)))
    return np.minimum(b, 30.0)


def synthetic_ocean(n=2048, dx=500.0, seed=3, amp=5.0, halfwidth=15e3,
                    centre=(650e3, 512e3), meander=20e3, meander_period=256e3,
                    roughness_std=50.0, alpha=3.0, steps=5000, ngauge_side=8,
                    cfl=0.9):
    """Synthetic ocean: abyssal plain with seeded roughness, continental slope,
    shelf and coastline (dry land up to +30 m); landslide-like dipole source
    eta' = -A sqrt(2e) s_x exp(-(s_x^2 + s_y^2)), s = (x - x_c)/halfwidth;
    extrapolation boundaries; fixed dt = cfl dx / max(Ce) at t = 0."""
    rng = np.random.default_rng(seed)
    L = n * dx
    grid = Grid(n, n, 0.0, 0.0, dx, dx, (BC_EXTRAP,) * 4)
    X, Y = cell_centres(grid)
    scale = L / 1024e3
    d = X + meander * scale * np.sin(2.0 * np.pi * Y / (meander_period * scale))
    b0 = _ocean_profile(d, L)
    noise = rng.standard_normal((n, n))
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=dx)
    KX, KY = np.meshgrid(k, k)
    sig = 5e3
    filt = np.exp(-0.5 * (KX ** 2 + KY ** 2) * sig ** 2)
    rough = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
    rough *= roughness_std / rough.std()
    f = d / L
    lo, hi = 580.0 / 1024.0, 620.0 / 1024.0
    taper = np.clip((hi - f) / (hi - lo), 0.0, 1.0)
    b = fp32_representable(b0 + rough * taper)
    sx = (X - centre[0] * scale) / halfwidth
    sy = (Y - centre[1] * scale) / halfwidth
    eta = -amp * math.sqrt(2.0 * math.e) * sx * np.exp(-(sx ** 2 + sy ** 2))
    h = np.maximum(eta - b, 0.0)
    h = np.where(b >= 0.0, 0.0, h)
    q = np.zeros((7, n, n))
    q[0] = h
    params = Params(alpha=alpha, h_star=20.0, kappa=0.8, dry_tol=1e-3, cfl=cfl)
    H = np.maximum(-b, 0.0)
    ce = np.sqrt(G * h + alpha * alpha * G * H)
    dt = cfl * dx / float(ce.max())
    gx = np.array([300, 500, 560, 620, 680, 760, 880, 940], dtype=float) * 1e3 * scale
    gy = np.array([128, 256, 384, 448, 576, 640, 768, 896], dtype=float) * 1e3 * scale
    gauges = np.array([[x, y] for x in gx[:ngauge_side] for y in gy[:ngauge_side]])
    return Workload("synthetic_ocean_%dx%d" % (n, n), params, grid, b, q, gauges,
                    steps, dt, amp)


def ensemble(count=48, seed0=5000, nmin=512, nmax=1536, steps=3000):
    """Ensemble of independent source scenarios: grid sides U{nmin..nmax},
    spacing U[500, 2000] m, the synthetic-ocean profile scaled to each domain,
    dipole amplitude U[1, 8] m, half-width U[5, 30] km at (0.635 L, 0.5 L),
    16 gauges per scenario on a 4 x 4 lattice in the wet region."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(seed0 + s)
        n = int(rng.integers(nmin, nmax + 1))
        dx = float(rng.uniform(500.0, 2000.0))
        amp = float(rng.uniform(1.0, 8.0))
        hw = float(rng.uniform(5e3, 30e3))
        L = n * dx
        w = synthetic_ocean(n=n, dx=dx, seed=seed0 + s, amp=amp, halfwidth=hw,
                            centre=(0.635 * 1024e3, 0.5 * 1024e3), steps=steps,
                            ngauge_side=0)
        gx = np.array([0.30, 0.40, 0.50, 0.58]) * L
        gy = np.array([0.2, 0.4, 0.6, 0.8]) * L
        w.gauges = np.array([[x, y] for x in gx for y in gy])
        w.name = "ensemble_%02d_%dx%d" % (s, n, n)
        out.append(w)
    return out


# --------------------------------------------------------------------------
# patch sets (static AMR)

@dataclasses.dataclass
class PatchSpec:
    level: int
    nx: int
    ny: int
    x0: float
    y0: float
    b: np.ndarray              # [ny, nx]
    q: np.ndarray              # [7, ny, nx]


@dataclasses.dataclass
class AmrWorkload:
    """One scenario on a static patch set: level-0 spacing dx0, dy0; level l
    has spacing dx0 / 4^l; `bc` applies on the domain boundary."""
    name: str
    params: Params
    dx0: float
    dy0: float
    bc: tuple
    patches: list
    gauges: np.ndarray
    steps: int
    dt: float                  # fixed level-0 step
    amplitude: float


RATIO = 4


def tiled(w: Workload, kx: int, ky: int) -> AmrWorkload:
    """A single-grid workload cut into kx x ky level-0 patches."""
    g = w.grid
    xs = np.linspace(0, g.nx, kx + 1).astype(int)
    ys = np.linspace(0, g.ny, ky + 1).astype(int)
    patches = []
    for j in range(ky):
        for i in range(kx):
            sl = (slice(ys[j], ys[j + 1]), slice(xs[i], xs[i + 1]))
            patches.append(PatchSpec(0, int(xs[i + 1] - xs[i]), int(ys[j + 1] - ys[j]),
                                     g.x0 + xs[i] * g.dx, g.y0 + ys[j] * g.dy,
                                     w.b[sl].copy(), w.q[(slice(None),) + sl].copy()))
    return AmrWorkload(w.name + "_tiled%dx%d" % (kx, ky), w.params, g.dx, g.dy, g.bc, patches,
                       w.gauges, w.steps, w.dt, w.amplitude)


def _ring_state(X, Y, b, centre, r0, width, amp, g=G):
    """outgoing circular long wave: eta' = A exp(-((r - r0)/w)^2), depth-
    averaged radial momentum eta' sqrt(g H), auxiliaries zero"""
    dxc, dyc = X - centre[0], Y - centre[1]
    r = np.sqrt(dxc ** 2 + dyc ** 2)
    eta = amp * np.exp(-((r - r0) / width) ** 2)
    H = np.maximum(-b, 0.0)
    h = np.maximum(eta - b, 0.0)
    h = np.where(b >= 0.0, 0.0, h)
    m = eta * np.sqrt(g * H)
    rr = np.where(r > 0, r, 1.0)
    q = np.zeros((7,) + X.shape)
    q[0] = h
    q[1] = np.where(h > 0, m * dxc / rr, 0.0)
    q[2] = np.where(h > 0, m * dyc / rr, 0.0)
    return q


def _bilinear(field, x0, y0, dx, X, Y):
    """bilinear interpolation of a cell-centred field (origin x0, y0) at
    points X, Y (clamped at the edges)"""
    ny, nx = field.shape
    fx = np.clip((X - x0) / dx - 0.5, 0.0, nx - 1.000001)
    fy = np.clip((Y - y0) / dx - 0.5, 0.0, ny - 1.000001)
    i0 = np.floor(fx).astype(int)
    j0 = np.floor(fy).astype(int)
    wx, wy = fx - i0, fy - j0
    return ((1 - wx) * (1 - wy) * field[j0, i0] + wx * (1 - wy) * field[j0, i0 + 1]
            + (1 - wx) * wy * field[j0 + 1, i0] + wx * wy * field[j0 + 1, i0 + 1])


def _basin(n0, dx, depth, amp, width, rough, seed):
    """bathymetry and initial state (functions of cell centres) of the small
    deep basin: depth plus four seeded smooth bumps, a Gaussian hump at rest
    centred at (0.45 L, 0.55 L)"""
    rng = np.random.default_rng(seed)
    L = n0 * dx
    bumps = rng.standard_normal((4, 3))

    def bath(X, Y):
        b = -depth + 0.0 * X
        for a, cx, cy in bumps:
            b = b + rough * a * np.exp(-(((X / L - 0.5 - 0.3 * cx) ** 2
                                          + (Y / L - 0.5 - 0.3 * cy) ** 2) / 0.02))
        return fp32_representable(b)

    def state(X, Y, b):
        eta = amp * np.exp(-(((X - 0.45 * L) ** 2 + (Y - 0.55 * L) ** 2) / width ** 2))
        q = np.zeros((7,) + X.shape)
        q[0] = np.maximum(eta - b, 0.0)
        return q

    return bath, state


def amr_small(n0=48, tiles=2, dx=500.0, depth=4000.0, amp=1.0, width=3e3,
              fine=((1, 64, 80, 40, 40), (1, 104, 88, 24, 32), (2, 300, 360, 48, 40)),
              bc=(BC_WALL,) * 4, steps=6, rough=200.0, seed=11, cfl=0.9):
    """Small three-level patch set: an n0 x n0 deep basin (depth plus seeded
    smooth roughness) in tiles x tiles level-0 patches, a Gaussian hump at
    rest off-centre, and the finer patches `fine` given as (level, i0, j0,
    nx, ny) in cells of their own level."""
    bath, state = _basin(n0, dx, depth, amp, width, rough, seed)
    L = n0 * dx
    patches = []
    cuts = np.linspace(0, n0, tiles + 1).astype(int)
    for j in range(tiles):
        for i in range(tiles):
            gx = Grid(int(cuts[i + 1] - cuts[i]), int(cuts[j + 1] - cuts[j]), cuts[i] * dx,
                      cuts[j] * dx, dx, dx, bc)
            X, Y = cell_centres(gx)
            b = bath(X, Y)
            patches.append(PatchSpec(0, gx.nx, gx.ny, gx.x0, gx.y0, b, state(X, Y, b)))
    for lev, i0, j0, nx, ny in fine:
        d = dx / RATIO ** lev
        gx = Grid(nx, ny, i0 * d, j0 * d, d, d, bc)
        X, Y = cell_centres(gx)
        b = bath(X, Y)
        patches.append(PatchSpec(lev, nx, ny, gx.x0, gx.y0, b, state(X, Y, b)))
    params = Params(alpha=3.0, h_star=20.0, kappa=0.8, dry_tol=1e-3, cfl=cfl)
    ce = math.sqrt(G * (depth + rough * 3 + amp) * (1 + 9.0))
    dt = cfl * dx / ce
    gauges = np.array([[0.45 * L, 0.55 * L], [0.3 * L, 0.3 * L], [0.62 * L, 0.5 * L],
                       [0.7 * L, 0.7 * L]])
    return AmrWorkload("amr_small_%d" % n0, params, dx, dx, bc, patches, gauges, steps, dt, amp)


def distortion(Lx, Ly, amp=0.005):
    """a smooth distortion of an Lx x Ly computational plane: each point
    moved by amp times the domain size along sine profiles (amp = 0.005:
    capacities within about 10% of 1)"""
    def f(XI, ETA):
        X = XI + amp * Lx * np.sin(2 * np.pi * ETA / Ly) * np.cos(2 * np.pi * XI / Lx)
        Y = ETA + amp * Ly * np.sin(2 * np.pi * XI / Lx) * np.sin(4 * np.pi * ETA / Ly)
        return X, Y
    return f


def distorted_nodes(g: Grid, amp=0.005):
    """nodes [ny + 5][nx + 5] (two ghost layers) of single grid g under
    distortion() of its own domain"""
    xi = g.x0 + np.arange(-2, g.nx + 3) * g.dx
    eta = g.y0 + np.arange(-2, g.ny + 3) * g.dy
    XI, ETA = np.meshgrid(xi, eta)
    return distortion(g.nx * g.dx, g.ny * g.dy, amp)(XI, ETA)


def distorted_patch_nodes(w: AmrWorkload, amp=0.005):
    """nodes of every patch of patch set w under distortion() of its level-0
    domain, finer levels by bilinear refinement (nested_nodes)"""
    lv0 = [p for p in w.patches if p.level == 0]
    Lx = max(p.x0 + p.nx * w.dx0 for p in lv0) - min(p.x0 for p in lv0)
    Ly = max(p.y0 + p.ny * w.dy0 for p in lv0) - min(p.y0 for p in lv0)
    return nested_nodes(w, distortion(Lx, Ly, amp))


def nested_nodes(w: AmrWorkload, fmap):
    """node coordinates of every patch of the patch set w under a mapping
    fmap(xi, eta) -> (x, y) of the level-0 computational plane: the level-0
    nodes (two ghost layers beyond the domain included) are fmap at the
    level-0 node positions; a level-l node is the bilinear interpolant of the
    four level-0 nodes around it, so that the nodes of each level are the
    bilinear refinement of the coarser level's and the fine cells tile each
    coarse cell exactly.  Returns [(xn, yn)] in patch order, each
    [ny + 5][nx + 5] (nodes i = -2..nx+2, j = -2..ny+2)."""
    lv0 = [p for p in w.patches if p.level == 0]
    X0, Y0 = min(p.x0 for p in lv0), min(p.y0 for p in lv0)
    NX = max(int(round((p.x0 - X0) / w.dx0)) + p.nx for p in lv0)
    NY = max(int(round((p.y0 - Y0) / w.dy0)) + p.ny for p in lv0)
    XI, ETA = np.meshgrid(X0 + np.arange(-2, NX + 3) * w.dx0, Y0 + np.arange(-2, NY + 3) * w.dy0)
    nx0, ny0 = fmap(XI, ETA)
    out = []
    for p in w.patches:
        r = RATIO ** p.level
        I0 = int(round((p.x0 - X0) / (w.dx0 / r)))
        J0 = int(round((p.y0 - Y0) / (w.dy0 / r)))
        # level-0 node coordinates (in nodes from node -2) of the patch's nodes
        fi = (I0 + np.arange(-2, p.nx + 3)) / r + 2.0
        fj = (J0 + np.arange(-2, p.ny + 3)) / r + 2.0
        ci = np.minimum(np.floor(fi).astype(int), NX + 3)
        cj = np.minimum(np.floor(fj).astype(int), NY + 3)
        ti, tj = fi - ci, fj - cj
        CI, CJ = np.meshgrid(ci, cj)
        TI, TJ = np.meshgrid(ti, tj)
        res = []
        for n in (nx0, ny0):
            res.append((n[CJ, CI] * (1.0 - TI) + n[CJ, CI + 1] * TI) * (1.0 - TJ)
                       + (n[CJ + 1, CI] * (1.0 - TI) + n[CJ + 1, CI + 1] * TI) * TJ)
        out.append(tuple(res))
    return out


def amr_small_uniform(level, n0=48, dx=500.0, depth=4000.0, amp=1.0, width=3e3,
                      bc=(BC_WALL,) * 4, steps=6, rough=200.0, seed=11, cfl=0.9):
    """The basin of amr_small on one uniform grid at the spacing of `level`,
    with 4^level steps of dt / 4^level per level-0 step"""
    bath, state = _basin(n0, dx, depth, amp, width, rough, seed)
    r = RATIO ** level
    grid = Grid(n0 * r, n0 * r, 0.0, 0.0, dx / r, dx / r, bc)
    X, Y = cell_centres(grid)
    b = bath(X, Y)
    w = amr_small(n0=n0, dx=dx, depth=depth, amp=amp, width=width, bc=bc, steps=steps,
                  rough=rough, seed=seed, cfl=cfl)
    return Workload("basin_uniform_level%d" % level, w.params, grid, b, state(X, Y, b), w.gauges,
                    steps * r, w.dt / r, amp)


def amr_ocean(n=2048, dx=500.0, tile=128, seed=4, targets=(1000, 1250),
              band=(40e3, 10e3), r0=430e3, ring_amp=0.5, ring_width=15e3,
              centre=(650e3, 512e3), max_tries=1_000_000, steps=500, cfl=0.9,
              deep=-1000.0):
    """Three-level patch set on the synthetic ocean: level 0 is the 2048^2
    ocean at 500 m cut into 128^2 patches; levels 1 (125 m) and 2 (31.25 m)
    hold patches with sides drawn from {16, 20, ..., 128} cells of their own
    level, placed by seeded rejection sampling in deep water around a ring of
    radius r0 about the source (half-widths band[0] and band[1]); level-2
    patches nest inside one level-1 patch shrunk by one level-1 cell.  The
    state is an outgoing circular long wave on that ring.  Fine bathymetry
    is the bilinear interpolation of the level-0 bathymetry."""
    base = synthetic_ocean(n=n, dx=dx, steps=steps, cfl=cfl)
    rng = np.random.default_rng(seed)
    L = n * dx
    scale = L / 1024e3
    c = (centre[0] * scale, centre[1] * scale)
    b0 = base.b
    patches = []
    for J in range(0, n, tile):
        for I in range(0, n, tile):
            g = Grid(tile, tile, I * dx, J * dx, dx, dx, base.grid.bc)
            X, Y = cell_centres(g)
            bb = b0[J:J + tile, I:I + tile].copy()
            patches.append(PatchSpec(0, tile, tile, g.x0, g.y0, bb,
                                     _ring_state(X, Y, bb, c, r0 * scale, ring_width, ring_amp)))
    sides = np.arange(16, 129, 4)

    def deep_enough(x0, y0, w, h):
        i0, j0 = int(x0 // dx), int(y0 // dx)
        i1, j1 = int(math.ceil((x0 + w) / dx)), int(math.ceil((y0 + h) / dx))
        if i0 < 1 or j0 < 1 or i1 > n - 1 or j1 > n - 1:
            return False
        return float(b0[j0:j1, i0:i1].max()) < deep

    # level 1: occupancy in level-1 cells
    d1 = dx / RATIO
    n1 = n * RATIO
    occ1 = np.zeros((n1, n1), dtype=bool)
    lev1 = []
    tries = 0
    while len(lev1) < targets[0] and tries < max_tries:
        tries += 1
        th = rng.uniform(0, 2 * math.pi)
        rr = r0 * scale + rng.uniform(-band[0], band[0])
        wx, wy = int(rng.choice(sides)), int(rng.choice(sides))
        cx, cy = c[0] + rr * math.cos(th), c[1] + rr * math.sin(th)
        i0 = int(round((cx / d1 - wx / 2) / RATIO)) * RATIO
        j0 = int(round((cy / d1 - wy / 2) / RATIO)) * RATIO
        if i0 < RATIO or j0 < RATIO or i0 + wx > n1 - RATIO or j0 + wy > n1 - RATIO:
            continue
        if occ1[j0:j0 + wy, i0:i0 + wx].any():
            continue
        if not deep_enough(i0 * d1, j0 * d1, wx * d1, wy * d1):
            continue
        occ1[j0:j0 + wy, i0:i0 + wx] = True
        lev1.append((i0, j0, wx, wy))
    # level 2: inside one level-1 patch shrunk by one level-1 cell
    d2 = d1 / RATIO
    lev2 = []
    occ2 = {}
    tries = 0
    while len(lev2) < targets[1] and tries < max_tries and lev1:
        tries += 1
        k = int(rng.integers(len(lev1)))
        pi0, pj0, pw, ph = lev1[k]
        wx, wy = int(rng.choice(sides)), int(rng.choice(sides))
        inner_w, inner_h = (pw - 2) * RATIO, (ph - 2) * RATIO     # in level-2 cells
        if wx > inner_w or wy > inner_h:
            continue
        ox = int(rng.integers(0, (inner_w - wx) // RATIO + 1)) * RATIO
        oy = int(rng.integers(0, (inner_h - wy) // RATIO + 1)) * RATIO
        o = occ2.setdefault(k, np.zeros((inner_h, inner_w), dtype=bool))
        if o[oy:oy + wy, ox:ox + wx].any():
            continue
        o[oy:oy + wy, ox:ox + wx] = True
        lev2.append(((pi0 + 1) * RATIO + ox, (pj0 + 1) * RATIO + oy, wx, wy))
    for lev, items, d in ((1, lev1, d1), (2, lev2, d2)):
        for i0, j0, wx, wy in items:
            g = Grid(wx, wy, i0 * d, j0 * d, d, d, base.grid.bc)
            X, Y = cell_centres(g)
            bb = fp32_representable(_bilinear(b0, 0.0, 0.0, dx, X, Y))
            patches.append(PatchSpec(lev, wx, wy, g.x0, g.y0, bb,
                                     _ring_state(X, Y, bb, c, r0 * scale, ring_width, ring_amp)))
    ang = np.linspace(0.55 * math.pi, 1.45 * math.pi, 16)
    gauges = np.array([[c[0] + r0 * scale * math.cos(a), c[1] + r0 * scale * math.sin(a)]
                       for a in ang])
    name = "amr_ocean_%d_L0x%d_L1x%d_L2x%d" % (n, (n // tile) ** 2, len(lev1), len(lev2))
    return AmrWorkload(name, base.params, dx, dx, base.grid.bc, patches, gauges, steps,
                       base.dt, ring_amp)
