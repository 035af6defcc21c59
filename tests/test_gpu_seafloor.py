"""GPU: the seafloor moving under a set state.  A bathymetry change between
steps generates the wave, as the sea-floor motion of the Tohoku case
(Sec. 6.4) does.  Every form keeps each cell's depth h under the new bottom,
so that the surface moves with the seafloor, as the oracle does (its state is
h, independent of b).

Bar: right after the change, FP64 depths equal the old ones exactly and mixed
ones within 1e-6 m.  After further steps, FP64 fields are within 1e-11 of the
oracle relative to each field's largest magnitude, and masks are equal.
Mixed gauges are within 1e-4 of the uplift amplitude of the FP64 run (deep
water; the rough wet/dry case checks FP64 parity and the kept depths).
"""
import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from cases import rough_case
from oracle.parity import oracle_bars

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11
UPLIFT = 2.0          # m


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def uplift(grid, b, amp, frac=(0.4, 0.45), width=0.15):
    """b raised by a Gaussian of height amp centred at frac of the domain,
    rounded to FP32-representable values"""
    X, Y = W.cell_centres(grid)
    Lx, Ly = grid.nx * grid.dx, grid.ny * grid.dy
    r2 = ((X - grid.x0 - frac[0] * Lx) / (width * Lx)) ** 2 + \
        ((Y - grid.y0 - frac[1] * Ly) / (width * Ly)) ** 2
    return W.fp32_representable(b + amp * np.exp(-r2))


def field_errors(got, exp):
    scale = np.abs(exp).max(axis=(1, 2))
    return np.abs(got - exp).max(axis=(1, 2)) / np.where(scale > 0, scale, 1.0)


@pytest.mark.parametrize("case", ["deep_basin", "rough_shore"])
def test_single_grid_seafloor_motion(case):
    if case == "deep_basin":
        w = W.amr_small_uniform(0, steps=4)
        w.b = W.fp32_representable(w.b)
        amp = UPLIFT
    else:
        w = rough_case(73, 41, (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), seed=5)
        amp = 0.05
    b1 = uplift(w.grid, w.b, amp)
    gauges = {}
    for precision in (0, 1):
        print("case", w.name, "precision", precision, flush=True)
        ctx = H.from_workloads([w], precision=precision)
        ctx.advance(w.dt, 3)
        h0 = ctx.get_state(0)[0]
        ctx.set_bathymetry(0, b1)
        h1 = ctx.get_state(0)[0]
        if precision == 0:
            assert np.array_equal(h0, h1)
        else:
            assert np.abs(h1 - h0).max() <= 1e-6
        ctx.advance(w.dt, 12)
        if precision == 0:
            r = O.from_workload(w)
            r.advance(w.dt, 3)
            r.set_bathymetry(b1)
            r.advance(w.dt, 12)
            err = field_errors(ctx.get_state(0), r.get_state())
            print("field errors", np.array2string(err, precision=2))
            assert np.all(err <= TOL)
            assert np.array_equal(ctx.get_mask(0), r.get_mask())
        gauges[precision] = ctx.read_gauges(0)[1]
        ctx.close()
    ge = np.abs(gauges[1] - gauges[0]).max() / amp
    print("mixed vs FP64 gauge error / uplift", ge)
    if case == "deep_basin":            # the rough shore's 0.1 m depths are below that bar
        assert ge <= 1e-4


def test_patch_set_seafloor_motion():
    """uplift under a level-0 patch and the level-1 patch inside it of the
    small three-level basin"""
    w = W.amr_small(steps=2)
    for p in w.patches:
        p.b[...] = W.fp32_representable(p.b)
    moved = {}
    for pid, p in enumerate(w.patches):
        d = w.dx0 / 4 ** p.level
        g = W.Grid(p.nx, p.ny, p.x0, p.y0, d, d, w.bc)
        full = W.Grid(48, 48, 0.0, 0.0, w.dx0, w.dy0, w.bc)
        X, Y = W.cell_centres(g)
        L = full.nx * full.dx
        bump = UPLIFT * np.exp(-(((X - 0.4 * L) / (0.12 * L)) ** 2 + ((Y - 0.45 * L) / (0.12 * L)) ** 2))
        moved[pid] = W.fp32_representable(p.b + bump)
    gauges = {}
    for precision in (0, 1):
        print("case", w.name, "precision", precision, flush=True)
        ctx, ids = H.from_amr_workloads([w], precision=precision)
        ctx.advance(-1.0, 1)
        h0 = [ctx.get_state(pid)[0] for pid in ids[0]]
        for pid in ids[0]:
            ctx.set_bathymetry(pid, moved[pid])
        for pid, h in zip(ids[0], h0):
            h1 = ctx.get_state(pid)[0]
            if precision == 0:
                assert np.array_equal(h, h1)
            else:
                assert np.abs(h1 - h).max() <= 1e-6
        ctx.advance(-1.0, 3)
        if precision == 0:
            runs = []

            def run(x):
                r = A.from_workload(x)
                r.advance(x.dt, 1)
                for k in range(len(x.patches)):
                    r.set_bathymetry(k, moved[k])
                r.advance(x.dt, 3)
                runs.append(r)
                return [r.get_state(k) for k in range(len(x.patches))]
            out, bars = oracle_bars(run, w)
            o = runs[0]
            for pid in ids[0]:
                err = field_errors(ctx.get_state(pid), out[pid])
                assert np.all(err <= bars[pid]), (pid, err, bars[pid])
                assert np.array_equal(ctx.get_mask(pid) & 3, o.get_mask(pid)), pid
        gauges[precision] = ctx.read_gauges(0)[1]
        ctx.close()
    ge = np.abs(gauges[1] - gauges[0]).max() / UPLIFT
    print("mixed vs FP64 gauge error / uplift", ge)
    assert ge <= 1e-4
