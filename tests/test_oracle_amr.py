"""Pins of the oracle's static patch sets (CPU only).

The paper gives no detail of its block-structured refinement beyond naming
the wave-propagation AMR of Berger and LeVeque (Sec. 4), so the rules are
readings; these tests pin what any correct implementation of them must
satisfy:
  * a level-0 tiling of one grid is the same computation as the grid itself
    (bitwise, every boundary condition, wet/dry);
  * a lake at rest over rough bathymetry stays exactly at rest through
    ghost interpolation, subcycling, refluxing and averaging down;
  * the mass of a closed basin is conserved to round-off with refluxing,
    and not without it (the planted variant shows the check is sharp);
  * refinement brings gauges closer to a uniformly fine solution.
"""
import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from paper_2606_12162_amd import workloads as W

from cases import rough_case


@pytest.mark.parametrize("bc, tiles", [
    ((W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), (3, 2)),
    ((W.BC_PERIODIC, W.BC_PERIODIC, W.BC_WALL, W.BC_EXTRAP), (2, 3)),
])
def test_level0_tiling_equals_single_grid_bitwise(bc, tiles):
    w = rough_case(61, 47, bc, seed=5)
    ref = O.from_workload(w)
    ref.advance(w.dt, 12)
    t = W.tiled(w, *tiles)
    o = A.from_workload(t)
    o.advance(w.dt, 12)
    q = ref.get_state()
    m = ref.get_mask()
    for pid, p in enumerate(t.patches):
        i0 = int(round(p.x0 / w.grid.dx))
        j0 = int(round(p.y0 / w.grid.dy))
        sl = (slice(j0, j0 + p.ny), slice(i0, i0 + p.nx))
        assert np.array_equal(o.get_state(pid), q[(slice(None),) + sl]), pid
        assert np.array_equal(o.get_mask(pid), m[sl]), pid
    # gauges whose 2 x 2 interpolation stencil lies inside one patch agree up
    # to the rounding of their weights (taken from the patch's own corner)
    _, eo = o.read_gauges()
    _, er = ref.read_gauges()
    inside = []
    for k, (x, y) in enumerate(w.gauges):
        i0 = int(np.floor(x / w.grid.dx - 0.5))
        j0 = int(np.floor(y / w.grid.dy - 0.5))
        for p in t.patches:
            pi0, pj0 = int(round(p.x0 / w.grid.dx)), int(round(p.y0 / w.grid.dy))
            if pi0 <= i0 and i0 + 1 < pi0 + p.nx and pj0 <= j0 and j0 + 1 < pj0 + p.ny:
                inside.append(k)
    assert inside
    assert np.abs(eo[:, inside] - er[:, inside]).max() <= 1e-14 * w.amplitude


def lake_at_rest(o):
    """set every patch to rest on the prepared bathymetry (covered coarse
    cells carry the mean of the fine bathymetry): h = -b, all else zero"""
    o.prepare()
    for pid, p in enumerate(o.patches):
        q = np.zeros((7, p.ny, p.nx))
        q[0] = np.maximum(-p.b[2:-2, 2:-2], 0.0)
        o.set_state(pid, q)


def test_lake_at_rest_is_exact_on_three_levels():
    w = W.amr_small(amp=0.0, steps=3)
    o = A.from_workload(w)
    lake_at_rest(o)
    o.advance(w.dt, w.steps)
    for pid, p in enumerate(o.patches):
        q = o.get_state(pid)
        b = p.b[2:-2, 2:-2]
        assert np.abs(q[1:]).max() == 0.0, pid
        assert np.array_equal(q[0], -b), pid


def test_mass_conserved_by_refluxing_and_lost_without_it():
    w = W.amr_small(steps=5)
    drift = {}
    for reflux in (True, False):
        o = A.from_workload(w, reflux=reflux)
        o.step(w.dt)                # the first step averages the fine start down
        m1 = o.mass()
        o.advance(w.dt, w.steps - 1)
        drift[reflux] = abs(o.mass() - m1) / m1
        assert o.clip == 0.0
    print("relative mass drift with / without refluxing", drift)
    assert drift[True] <= 2e-15
    assert drift[False] >= 1e-10


def test_refinement_approaches_the_fine_solution():
    """gauge 0 sits at the hump centre inside a level-1 patch: after 6 level-0
    steps the patch set is about 4 times closer to a uniform level-1 grid
    than the level-0 grid alone is (a wrong interpolation offset, time
    weight or reflux sign makes it worse than the coarse grid)"""
    steps = 6
    w = W.amr_small(steps=steps)
    o = A.from_workload(w)
    o.advance(w.dt, steps)
    _, e_amr = o.read_gauges()
    coarse = W.amr_small_uniform(0, steps=steps)
    fine = W.amr_small_uniform(1, steps=steps)
    rc = O.from_workload(coarse)
    rc.advance(coarse.dt, steps)
    rf = O.from_workload(fine)
    rf.advance(fine.dt, fine.steps)
    _, e_c = rc.read_gauges()
    _, e_f = rf.read_gauges()
    e_f = e_f[W.RATIO - 1::W.RATIO]          # the records at level-0 times
    err_amr = np.abs(e_amr[:, 0] - e_f[:, 0]).max()
    err_c = np.abs(e_c[:, 0] - e_f[:, 0]).max()
    print("gauge 0 distance to the fine grid: patch set %.3e, coarse grid %.3e" % (err_amr, err_c))
    assert err_amr < 0.35 * err_c


def test_ghost_interpolation_is_exact_for_linear_data():
    """coarse states linear in x and y at the old and new time levels: every
    level-1 ghost cell filled from level 0 equals the linear function at the
    ghost centre, blended in time with weight theta (minmod keeps the slope
    of linear data; the offsets are +-1/8 and +-3/8 of a coarse cell)"""
    w = W.amr_small(steps=1)
    o = A.from_workload(w)
    o.prepare()
    theta = 0.25
    co = np.array([[0.3, 2e-5, -1e-5], [5.0, 1e-3, 2e-3], [-2.0, 3e-4, 1e-4], [0.1, 0, 1e-6],
                   [0.2, 1e-6, 0], [50.0, 1e-2, -2e-2], [70.0, -1e-2, 3e-2]])
    cn = co * np.array([1.5, 0.5, 2.0])
    for p in o.levels[0]:
        X = p.x0 + (np.arange(-2, p.nx + 2) + 0.5) * p.dx
        Y = p.y0 + (np.arange(-2, p.ny + 2) + 0.5) * p.dy
        XX, YY = np.meshgrid(X, Y)
        old = np.empty_like(p.q)
        for m in range(7):
            old[m] = co[m, 0] + co[m, 1] * XX + co[m, 2] * YY
            p.q[m] = cn[m, 0] + cn[m, 1] * XX + cn[m, 2] * YY
        old[0] = old[0] - p.b          # plane 0 holds h; eta' is linear
        p.q[0] = p.q[0] - p.b
        o.old[p.pid] = old
    o.fill_ghosts(1, theta)
    checked = 0
    for f in o.levels[1]:
        for i, j in o._ghost_cells(f):
            src = o._source_of(f, i, j)
            if src[0] != "coarse":
                continue
            x = f.x0 + (i + 0.5) * f.dx
            y = f.y0 + (j + 0.5) * f.dy
            lin = [(1 - theta) * (co[m, 0] + co[m, 1] * x + co[m, 2] * y)
                   + theta * (cn[m, 0] + cn[m, 1] * x + cn[m, 2] * y) for m in range(7)]
            got = f.q[:, j + 2, i + 2].copy()
            got[0] = got[0] + f.b[j + 2, i + 2]
            np.testing.assert_allclose(got, lin, rtol=1e-12, atol=1e-9)
            checked += 1
    assert checked > 100
