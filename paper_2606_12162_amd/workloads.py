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
