"""Pins of the oracle's sponge layer (CPU only).

The Tohoku case (Sec. 6.4) damps reflections with a scalar relaxation sponge
whose form is cited, not described.  The reading: in a band of width w along
a chosen side of the domain, every conserved variable relaxes towards the
state at rest (h = H, the rest zero) by an implicit Euler step of rate
sigma = rate ((w - d) / w)^2, d being the cell centre's distance from that
side, after the second source half step and before the fix-ups.

Checked against what the reading and the scheme fix, not against the oracle:
  * one step from a uniform surface offset over a flat bottom (no fluxes, no
    source) gives h = H + eps / (1 + dt sigma) exactly, cell by cell, for
    four different widths on the four sides (a swapped side, a linear instead
    of a quadratic profile, or an explicit instead of implicit step fails);
  * a zero rate, or zero widths, changes no bit;
  * the sponge acts only in its band: after n steps the cells more than 2 n
    cells away from it are bitwise those of the run without it;
  * a wave running into a wall behind a sponge comes back with a small
    fraction of the energy that the bare wall reflects;
  * a patch set tiling a grid, sponge included, equals the single grid
    bitwise (the sponge's place in the domain is global, not per patch).
"""
import dataclasses

import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from paper_2606_12162_amd import workloads as W

from cases import rough_case


def flat_offset(nx=40, ny=30, dx=10.0, dy=12.0, depth=10.0, eps=0.01):
    grid = W.Grid(nx, ny, 0.0, 0.0, dx, dy, (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC))
    b = np.full((ny, nx), -depth)
    q = np.zeros((7, ny, nx))
    q[0] = depth + eps
    P = W.Params(alpha=3.0, h_star=0.0, kappa=0.8)
    return W.Workload("flat_offset", P, grid, b, q, np.zeros((0, 2)), 1, 0.05, eps)


def test_one_step_from_a_uniform_offset_is_the_closed_form():
    w = flat_offset()
    widths, rate, dt = (55.0, 35.0, 24.0, 30.0), 0.7, 0.05
    r = O.from_workload(w)
    r.set_sponge(widths, rate)
    r.advance(dt, 1)
    q = r.get_state()
    g = w.grid
    x = (np.arange(g.nx) + 0.5) * g.dx
    y = (np.arange(g.ny) + 0.5) * g.dy
    X, Y = np.meshgrid(x, y)
    d = [X, g.nx * g.dx - X, Y, g.ny * g.dy - Y]
    s = np.zeros_like(X)
    for wd, dd in zip(widths, d):
        s = np.maximum(s, np.where(dd < wd, (wd - dd) / wd, 0.0))
    expected = 10.0 + 0.01 / (1.0 + dt * rate * s * s)
    assert np.abs(q[0] - expected).max() <= 1e-14
    assert np.abs(q[1:]).max() == 0.0
    assert (s > 0).sum() > 0.3 * s.size          # the bands cover a good part of the grid


@pytest.mark.parametrize("widths,rate", [((0.0, 0.0, 0.0, 0.0), 0.5), ((0.3, 0.2, 0.4, 0.5), 0.0)])
def test_no_sponge_changes_no_bit(widths, rate):
    w = rough_case(41, 33, (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), seed=3)
    w = dataclasses.replace(w, gauges=np.zeros((0, 2)))
    a = O.from_workload(w)
    a.advance(w.dt, 10)
    b = O.from_workload(w)
    b.set_sponge(widths, rate)
    b.advance(w.dt, 10)
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.get_mask(), b.get_mask())


def test_sponge_acts_only_in_its_band():
    w = rough_case(61, 33, (W.BC_WALL, W.BC_EXTRAP, W.BC_WALL, W.BC_WALL), seed=4)
    w = dataclasses.replace(w, gauges=np.zeros((0, 2)))
    nsteps, band = 6, 8                         # band: cells from the x-high side
    a = O.from_workload(w)
    a.advance(w.dt, nsteps)
    b = O.from_workload(w)
    b.set_sponge((0.0, band * w.grid.dx, 0.0, 0.0), 2.0)
    b.advance(w.dt, nsteps)
    qa, qb = a.get_state(), b.get_state()
    far = w.grid.nx - band - 2 * nsteps        # the dependence spreads 2 cells a step
    assert np.array_equal(qa[:, :, :far], qb[:, :, :far])
    assert not np.array_equal(qa[:, :, far:], qb[:, :, far:])


def channel_energy_after_reflection(sponge):
    nx, ny, dx, depth = 300, 4, 1.0, 1.0
    grid = W.Grid(nx, ny, 0.0, 0.0, dx, dx, (W.BC_WALL, W.BC_WALL, W.BC_PERIODIC, W.BC_PERIODIC))
    X, _ = W.cell_centres(grid)
    b = np.full((ny, nx), -depth)
    q = np.zeros((7, ny, nx))
    eta = 0.01 * np.exp(-((X - 150.0) / 6.0) ** 2)
    q[0] = depth + eta
    c = np.sqrt(W.G * depth)
    q[1] = q[0] * c * eta / depth               # right-going long wave
    P = W.Params(alpha=3.0, h_star=0.0, kappa=0.0)
    dt = 0.45 * dx / (c * np.sqrt(1 + 9.0))
    wl = W.Workload("channel", P, grid, b, q, np.zeros((0, 2)), 1, dt, 0.01)
    r = O.from_workload(wl)
    if sponge:
        r.set_sponge((0.0, 60.0, 0.0, 0.0), 2.0)
    # the hump runs 150 m to the wall and 230 m back, into the left half
    r.advance(dt, int(round(380.0 / c / dt)))
    s = r.get_state()
    left = s[:, :, :150]
    return float(((left[0] - depth) ** 2).sum() + (left[1] ** 2 / (W.G * depth ** 2 / depth)).sum())


def test_sponge_absorbs_a_wave_that_a_wall_reflects():
    bare = channel_energy_after_reflection(False)
    damped = channel_energy_after_reflection(True)
    print("energy back in the left half: wall %.3e, wall behind the sponge %.3e" % (bare, damped))
    assert damped < 0.05 * bare


def test_patch_set_tiling_equals_single_grid_with_sponge():
    w = rough_case(61, 47, (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), seed=6)
    widths, rate = (0.6, 0.9, 0.0, 1.2), 3.0
    ref = O.from_workload(w)
    ref.set_sponge(widths, rate)
    ref.advance(w.dt, 10)
    t = W.tiled(w, 3, 2)
    o = A.from_workload(t)
    o.set_sponge(widths, rate)
    o.advance(w.dt, 10)
    q = ref.get_state()
    for pid, p in enumerate(t.patches):
        i0 = int(round(p.x0 / w.grid.dx))
        j0 = int(round(p.y0 / w.grid.dy))
        sl = (slice(None), slice(j0, j0 + p.ny), slice(i0, i0 + p.nx))
        assert np.array_equal(o.get_state(pid), q[sl]), pid
