"""Pins of the oracle's mapped patch sets (CPU only).

A mapped patch set runs the mapped-grid scheme of Sec. 4 on every patch of
a static patch set: fine nodes are the bilinear refinement of the coarse
ones, refluxing divides by the coarse capacity, averaging down weighs the
fine cells by their capacities, level-0 walls mirror the momentum about the
wall edge, and the coarse-fine flux records are solved in the fine edges'
frames.  What the geometry and the Cartesian rules fix, checked here without
using the oracle as its own reference:

  * the identity mapping gives the Cartesian patch set bitwise (three
    levels, walls);
  * a level-0 tiling of a rotated, distorted grid is the single mapped grid
    bitwise (every boundary condition, wet/dry): ghost copies and the wall
    mirror are the single grid's;
  * a patch set whose nodes are turned by 90 degrees about the origin
    (exact in binary), with its momenta turned, gives the turned solution:
    bitwise on a straight grid, to round-off on a distorted one.  A flux
    record solved in the Cartesian frame instead of the fine edge's fails
    it (planted below).  Other angles are not covariant under the rules,
    because the ghost interpolation limits hu and hv one by one (minmod
    commutes with a quarter turn, not with a general rotation);
  * the capacity-weighted mass of a distorted periodic patch set is
    conserved to round-off, and not without the capacities (planted);
  * a lake at rest over rough bathymetry on a distorted three-level set
    stays exactly at rest;
  * the nested nodes tile: the fine capacities of a coarse cell sum to 16
    times its capacity, to the rounding of the areas.
"""
import dataclasses

import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from paper_2606_12162_amd import workloads as W

from cases import rough_case

L48 = 48 * 500.0          # side of the amr_small basin (m)


def identity(x, y):
    return x, y


def bumpy(Lx, Ly, amp=0.04):
    """a smooth distortion vanishing on the sides of an Lx x Ly box"""
    def f(x, y):
        return (x + amp * Lx * np.sin(2 * np.pi * x / Lx) * np.sin(np.pi * y / Ly),
                y - 0.75 * amp * Ly * np.sin(np.pi * x / Lx) * np.sin(2 * np.pi * y / Ly))
    return f


def periodic_bumpy(Lx, Ly, amp=0.04):
    """a smooth distortion periodic over an Lx x Ly box"""
    def f(x, y):
        s = np.sin(2 * np.pi * x / Lx) * np.sin(2 * np.pi * y / Ly)
        return x + amp * Lx * s, y - 0.75 * amp * Ly * s
    return f


def turned(f, th):
    """f followed by a rotation by th about the origin"""
    c, s = np.cos(th), np.sin(th)

    def g(x, y):
        X, Y = f(x, y)
        return c * X - s * Y, s * X + c * Y
    return g


def quarter(f):
    """f followed by a quarter turn about the origin, exact in binary"""
    def g(x, y):
        X, Y = f(x, y)
        return 0.0 - Y, X
    return g


def with_momentum(w):
    """the basin of w with smooth momenta (the start at rest has none)"""
    ps = []
    for p in w.patches:
        d = w.dx0 / W.RATIO ** p.level
        X, Y = np.meshgrid(p.x0 + (np.arange(p.nx) + 0.5) * d, p.y0 + (np.arange(p.ny) + 0.5) * d)
        q = p.q.copy()
        q[1] = q[0] * 0.2 * np.sin(2 * np.pi * X / L48) * np.cos(np.pi * Y / L48)
        q[2] = q[0] * 0.15 * np.cos(np.pi * X / L48) * np.sin(2 * np.pi * Y / L48)
        ps.append(dataclasses.replace(p, q=q))
    return dataclasses.replace(w, patches=ps)


def quarter_state(q):
    """momenta turned by a quarter: (hu, hv) -> (-hv, hu)"""
    r = q.copy()
    r[1], r[2] = 0.0 - q[2], q[1]
    return r


def run(w, fmap, steps, dt_scale=0.7, **kw):
    o = A.from_workload(w, nodes=W.nested_nodes(w, fmap), **kw)
    o.advance(dt_scale * w.dt, steps)
    return o


def test_identity_mapping_is_the_cartesian_patch_set_bitwise():
    w = with_momentum(W.amr_small(steps=3))
    a = A.from_workload(w)
    a.advance(w.dt, 3)
    b = run(w, identity, 3, dt_scale=1.0)
    for k in range(len(w.patches)):
        assert np.array_equal(a.get_state(k), b.get_state(k)), k
        assert np.array_equal(a.get_mask(k), b.get_mask(k)), k
    assert a.mass() == b.mass()


@pytest.mark.parametrize("bc, tiles", [
    ((W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), (3, 2)),
    ((W.BC_WALL, W.BC_WALL, W.BC_WALL, W.BC_EXTRAP), (2, 3)),
])
def test_level0_tiling_is_the_single_mapped_grid_bitwise(bc, tiles):
    w = rough_case(61, 47, bc, seed=5)
    g = w.grid
    fmap = turned(bumpy(g.nx * g.dx, g.ny * g.dy, amp=0.02), 0.6)
    xi = g.x0 + np.arange(-2, g.nx + 3) * g.dx
    eta = g.y0 + np.arange(-2, g.ny + 3) * g.dy
    XI, ETA = np.meshgrid(xi, eta)
    ref = O.from_workload(w)
    ref.set_mapping(*fmap(XI, ETA))
    dt = 0.8 * w.dt
    ref.advance(dt, 12)
    t = W.tiled(w, *tiles)
    o = A.from_workload(t, nodes=W.nested_nodes(t, fmap))
    o.advance(dt, 12)
    q, m = ref.get_state(), ref.get_mask()
    for pid, p in enumerate(t.patches):
        i0, j0 = int(round(p.x0 / g.dx)), int(round(p.y0 / g.dy))
        sl = (slice(j0, j0 + p.ny), slice(i0, i0 + p.nx))
        assert np.array_equal(o.get_state(pid), q[(slice(None),) + sl]), pid
        assert np.array_equal(o.get_mask(pid), m[sl]), pid
    assert abs(o.mass() - ref.mass()) <= 1e-14 * ref.mass()


def quarter_turn_errors(base, dflux=None, monkeypatch=None):
    w = with_momentum(W.amr_small(steps=3))
    wq = dataclasses.replace(w, patches=[dataclasses.replace(p, q=quarter_state(p.q))
                                         for p in w.patches])
    a = run(w, base, 3)
    if dflux is not None:
        monkeypatch.setattr(O, "edge_dflux_mapped_n", dflux)
    b = run(wq, quarter(base), 3)
    err, scale, bits = np.zeros(7), np.zeros(7), True
    for k in range(len(w.patches)):
        qa, qb = quarter_state(a.get_state(k)), b.get_state(k)
        bits = bits and np.array_equal(qa, qb) and np.array_equal(a.get_mask(k), b.get_mask(k))
        bk = a.patches[k].b[2:-2, 2:-2]
        qa[0] += bk                      # compare the surface, not the depth
        qb = qb.copy()
        qb[0] += bk
        err = np.maximum(err, np.abs(qa - qb).max(axis=(1, 2)))
        scale = np.maximum(scale, np.abs(qa).max(axis=(1, 2)))
    return bits, err / np.where(scale > 0, scale, 1.0)


def test_quarter_turn_of_a_straight_patch_set_is_bitwise():
    bits, err = quarter_turn_errors(identity)
    assert bits, err


def test_quarter_turn_of_a_distorted_patch_set():
    bits, err = quarter_turn_errors(bumpy(L48, L48))
    print("quarter turn, distorted: relative field errors", np.array2string(err, precision=2))
    assert np.all(err <= 1e-11)


def test_quarter_turn_notices_a_flux_record_in_the_wrong_frame(monkeypatch):
    """planted in the oracle: the coarse-fine flux records solved in the
    Cartesian frame (length ratio kept) instead of the fine edge's"""
    def cartesian(params, direction, qL, qR, bL, bR, c2L, c2R, nx, ny, gm):
        return O.edge_dflux_n(params, direction, qL, qR, bL, bR, c2L, c2R) * np.asarray(gm)[:, None]
    bits, err = quarter_turn_errors(identity, cartesian, monkeypatch)
    print("planted Cartesian-frame records: relative field errors", np.array2string(err, precision=2))
    assert not bits and err.max() >= 1e-6


def test_mass_conserved_with_capacities_and_lost_without():
    w = W.amr_small(steps=5, bc=(W.BC_PERIODIC,) * 4)
    nodes = W.nested_nodes(w, periodic_bumpy(L48, L48))
    drift = {}
    for cap in (True, False):
        o = A.from_workload(w, nodes=nodes, capacity=cap)
        o.step(0.7 * w.dt)          # the first step averages the fine start down
        m1 = o.mass()
        o.advance(0.7 * w.dt, w.steps - 1)
        drift[cap] = abs(o.mass() - m1) / m1
        assert o.clip == 0.0
    print("relative mass drift with / without capacities", drift)
    assert drift[True] <= 2e-15
    assert drift[False] >= 1e-10


def test_mass_with_walls_drifts_as_on_a_single_mapped_grid():
    """walls on a distorted grid mirror about a skew normal, which rounds:
    the patch set drifts no more than the single grid of its level 0"""
    w = W.amr_small(steps=5)
    f = bumpy(L48, L48)
    o = A.from_workload(w, nodes=W.nested_nodes(w, f))
    o.step(0.7 * w.dt)
    m1 = o.mass()
    o.advance(0.7 * w.dt, 4)
    drift = abs(o.mass() - m1) / m1
    u = W.amr_small_uniform(0, steps=5)
    xi = u.grid.x0 + np.arange(-2, u.grid.nx + 3) * u.grid.dx
    g = O.from_workload(u)
    g.set_mapping(*f(*np.meshgrid(xi, xi)))
    g.advance(0.7 * u.dt, 1)
    g1 = g.mass()
    g.advance(0.7 * u.dt, 4)
    ref = abs(g.mass() - g1) / g1
    print("mass drift: patch set %.2e, single grid %.2e" % (drift, ref))
    assert drift <= max(2.0 * ref, 1e-15) and drift <= 1e-13


def test_lake_at_rest_is_exact_on_a_distorted_three_level_set():
    w = W.amr_small(amp=0.0, steps=3)
    o = A.from_workload(w, nodes=W.nested_nodes(w, bumpy(L48, L48)))
    o.prepare()
    for pid, p in enumerate(o.patches):
        q = np.zeros((7, p.ny, p.nx))
        q[0] = np.maximum(-p.b[2:-2, 2:-2], 0.0)
        o.set_state(pid, q)
    o.advance(0.7 * w.dt, 3)
    for pid, p in enumerate(o.patches):
        q = o.get_state(pid)
        assert np.abs(q[1:]).max() == 0.0, pid
        assert np.array_equal(q[0], -p.b[2:-2, 2:-2]), pid


def test_nested_nodes_tile_the_coarse_cells():
    w = W.amr_small(steps=1)
    o = A.from_workload(w, nodes=W.nested_nodes(w, turned(bumpy(L48, L48), 0.3)))
    worst = 0.0
    for f in o.patches:
        if f.level == 0:
            continue
        nbx, nby = f.nx // W.RATIO, f.ny // W.RATIO
        s = np.zeros((nby, nbx))
        for a in range(W.RATIO):
            for b in range(W.RATIO):
                s += f.met[0][2 + a:2 + a + W.RATIO * nby:W.RATIO, 2 + b:2 + b + W.RATIO * nbx:W.RATIO]
        for c in o.levels[f.level - 1]:
            Ic0, Jc0 = f.I0 // W.RATIO, f.J0 // W.RATIO
            i0, i1 = max(Ic0, c.I0), min(Ic0 + nbx, c.I0 + c.nx)
            j0, j1 = max(Jc0, c.J0), min(Jc0 + nby, c.J0 + c.ny)
            if i0 >= i1 or j0 >= j1:
                continue
            kc = c.met[0][j0 - c.J0 + 2:j1 - c.J0 + 2, i0 - c.I0 + 2:i1 - c.I0 + 2]
            worst = max(worst, float(np.abs(kc - s[j0 - Jc0:j1 - Jc0, i0 - Ic0:i1 - Ic0] / 16).max()))
    print("max |kap_c - sum kap_f / 16|", worst)
    assert worst <= 1e-13


def test_a_patch_set_mapped_in_part_is_refused():
    w = W.amr_small(steps=1)
    nodes = W.nested_nodes(w, identity)
    o = A.from_workload(w)
    o.set_mapping(0, *nodes[0])
    with pytest.raises(ValueError):
        o.step(w.dt)
