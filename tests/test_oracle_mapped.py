"""Pins of the oracle's mapped grids (CPU only).

Sec. 4 extends the scheme to mapped (logically rectangular) grids by the
cited treatment of quadrilateral grids: each edge's Riemann problem is
solved in the frame of its normal, its waves, speeds and fluctuations are
scaled by the edge's length ratio, and each cell's update is divided by its
capacity (area ratio).  The oracle's reading, checked here against what the
geometry and the scheme fix, not against the oracle itself:

  * the identity mapping of a Cartesian grid (dyadic spacings, so that node
    differences, lengths and areas are exact) gives the Cartesian grid's
    bits, on wet/dry data with walls, extrapolation and periodic sides;
  * a grid scaled by powers of two along each axis gives the Cartesian grid
    of the scaled spacings bitwise (capacity sx sy, length ratios sy on the
    left edges and sx on the bottom ones; a ratio on the wrong edges, a
    missing capacity in the corrections, the transverse weights or the
    Courant number fails it);
  * a rotated grid, with the initial momenta rotated, gives the rotated
    solution (a wrong frame, sign or back-rotation fails it);
  * on a smoothly distorted periodic grid the capacity-weighted mass
    sum(kap h) dx dy is conserved (the fluctuations telescope only if the
    edge-length-weighted normals of each closed cell sum to zero: a wrong
    normal or length ratio fails it), a lake at rest over a rough bottom
    stays at rest exactly, and a uniform flow stays uniform (equal states
    give no waves in the fluctuation form).
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_12162_amd import workloads as W

from cases import rough_case

BCS = [(W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC),
       (W.BC_WALL, W.BC_WALL, W.BC_WALL, W.BC_EXTRAP)]


def nodes(g, fx, fy):
    """node coordinates [ny + 5][nx + 5] of the nodes (i, j), i = -2..nx+2,
    j = -2..ny+2, from computational node positions xi, eta"""
    xi = g.x0 + np.arange(-2, g.nx + 3) * g.dx
    eta = g.y0 + np.arange(-2, g.ny + 3) * g.dy
    XI, ETA = np.meshgrid(xi, eta)
    return fx(XI, ETA), fy(XI, ETA)


def dyadic_case(bc, seed, dx=0.125, dy=0.0625):
    w = rough_case(48, 40, bc, seed)
    grid = W.Grid(48, 40, 0.0, 0.0, dx, dy, bc)
    return dataclasses.replace(w, grid=grid, gauges=np.zeros((0, 2)))


@pytest.mark.parametrize("bc", BCS)
def test_identity_mapping_is_the_cartesian_grid_bitwise(bc):
    w = dyadic_case(bc, seed=11)
    a = O.from_workload(w)
    a.advance(w.dt, 12)
    b = O.from_workload(w)
    b.set_mapping(*nodes(w.grid, lambda x, y: x, lambda x, y: y))
    b.advance(w.dt, 12)
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.get_mask(), b.get_mask())
    assert a.mass() == b.mass()


@pytest.mark.parametrize("sx,sy", [(2.0, 0.5), (2.0, 2.0), (0.5, 4.0)])
@pytest.mark.parametrize("bc", BCS)
def test_scaled_grid_is_the_cartesian_grid_of_scaled_spacing(bc, sx, sy):
    w = dyadic_case(bc, seed=12)
    g = w.grid
    cart = dataclasses.replace(w, grid=W.Grid(g.nx, g.ny, 0.0, 0.0, sx * g.dx, sy * g.dy, bc))
    dt = w.dt * min(sx, sy)
    a = O.from_workload(cart)
    a.advance(dt, 10)
    b = O.from_workload(w)
    b.set_mapping(*nodes(g, lambda x, y: sx * x, lambda x, y: sy * y))
    b.advance(dt, 10)
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.get_mask(), b.get_mask())
    assert b.mass() == a.mass()


@pytest.mark.parametrize("bc", [BCS[0], (W.BC_WALL, W.BC_WALL, W.BC_PERIODIC, W.BC_PERIODIC)])
def test_rotated_grid_gives_the_rotated_solution(bc):
    w = rough_case(40, 36, bc, seed=13)
    w = dataclasses.replace(w, gauges=np.zeros((0, 2)))
    th = 0.6
    c, s = np.cos(th), np.sin(th)
    a = O.from_workload(w)
    a.advance(w.dt, 12)
    qa = a.get_state()
    q0 = w.q.copy()
    q0[1], q0[2] = c * w.q[1] - s * w.q[2], s * w.q[1] + c * w.q[2]
    b = O.from_workload(dataclasses.replace(w, q=q0))
    b.set_mapping(*nodes(w.grid, lambda x, y: c * x - s * y, lambda x, y: s * x + c * y))
    b.advance(w.dt, 12)
    qb = b.get_state()
    back = qb.copy()
    back[1], back[2] = c * qb[1] + s * qb[2], -s * qb[1] + c * qb[2]
    scale = np.abs(qa).max(axis=(1, 2))
    err = np.abs(back - qa).max(axis=(1, 2)) / np.where(scale > 0, scale, 1.0)
    print("rotated grid, relative field errors", np.array2string(err, precision=2))
    assert np.all(err <= 1e-10)
    assert np.array_equal(a.get_mask(), b.get_mask())
    assert not np.array_equal(qb[1], qa[1])      # the momenta really are rotated


def distorted(g, amp=0.03):
    """a smooth periodic distortion of the unit-period computational grid"""
    Lx, Ly = g.nx * g.dx, g.ny * g.dy
    fx = lambda x, y: x + amp * Lx * np.sin(2 * np.pi * y / Ly) * np.cos(2 * np.pi * x / Lx)
    fy = lambda x, y: y + amp * Ly * np.sin(2 * np.pi * x / Lx) * np.sin(4 * np.pi * y / Ly)
    return nodes(g, fx, fy)


def periodic_case(q, b, dt=0.005, nx=40, ny=32):
    bc = (W.BC_PERIODIC,) * 4
    grid = W.Grid(nx, ny, 0.0, 0.0, 0.2, 0.25, bc)
    P = W.Params(alpha=3.0, h_star=0.0, kappa=0.0)
    return W.Workload("periodic_%dx%d" % (nx, ny), P, grid, b, q, np.zeros((0, 2)), 1, dt, 0.1)


def test_uniform_flow_stays_uniform_on_a_distorted_grid():
    nx, ny = 40, 32
    q = np.zeros((7, ny, nx))
    q[0], q[1], q[2] = 1.0, 0.3, -0.2
    w = periodic_case(q, np.full((ny, nx), -1.0))
    r = O.from_workload(w)
    r.set_mapping(*distorted(w.grid))
    r.advance(w.dt, 20)
    dev = np.abs(r.get_state() - q).max(axis=(1, 2))
    print("uniform flow, max deviation per field", np.array2string(dev, precision=2))
    assert dev.max() <= 1e-13


def test_capacity_weighted_mass_is_conserved_and_the_mapping_matters():
    nx, ny = 40, 32
    g = periodic_case(np.zeros((7, ny, nx)), np.zeros((ny, nx))).grid
    X, Y = W.cell_centres(g)
    q = np.zeros((7, ny, nx))
    q[0] = 1.0 + 0.1 * np.exp(-((X - 4.0) ** 2 + (Y - 4.0) ** 2))
    q[1] = 0.05 * q[0]
    w = periodic_case(q, np.full((ny, nx), -1.0))
    r = O.from_workload(w)
    r.set_mapping(*distorted(g))
    m0 = r.mass()
    r.advance(w.dt, 40)
    rel = abs(r.mass() - m0) / m0
    print("mass drift", rel)
    assert rel <= 1e-13
    c = O.from_workload(w)
    c.advance(w.dt, 40)
    assert np.abs(c.get_state()[0] - r.get_state()[0]).max() > 1e-4


def test_lake_at_rest_over_a_rough_bottom_on_a_distorted_grid():
    nx, ny = 40, 32
    rng = np.random.default_rng(14)
    b = W.fp32_representable(-1.0 - 0.3 * rng.random((ny, nx)))
    q = np.zeros((7, ny, nx))
    q[0] = -b
    w = periodic_case(q, b)
    r = O.from_workload(w)
    r.set_mapping(*distorted(w.grid))
    r.advance(w.dt, 20)
    s = r.get_state()
    assert np.abs(s[0] + b).max() <= 1e-15
    assert np.abs(s[1:]).max() == 0.0


def test_bad_mappings_are_refused():
    w = dyadic_case(BCS[0], seed=15)
    r = O.from_workload(w)
    xn, yn = nodes(w.grid, lambda x, y: x, lambda x, y: y)
    with pytest.raises(Exception):
        r.set_mapping(-xn, yn)                       # clockwise cells: negative areas
    xn2 = xn.copy()
    xn2[5, 5] = xn2[5, 6]                            # a zero-length edge
    yn2 = yn.copy()
    yn2[5, 5] = yn2[5, 6]
    with pytest.raises(Exception):
        r.set_mapping(xn2, yn2)
