"""GPU parity of the sponge layer (the relaxation sponge of Sec. 6.4, as read
in the oracle: implicit relaxation towards the state at rest in bands along
chosen sides of the domain) through the C ABI.

Bar: FP64 fields within 1e-11 of the oracle relative to each field's largest
magnitude (on the deep basin: or within ten times the oracle's own spread
under one-ulp changes of the depths, parity.py), masks equal, on a wet/dry
single grid, a three-level patch set and
a patch set regridded under its sponge; mixed gauges within 1e-4 of the
amplitude of the FP64 run; bad widths and rates refused.
"""
import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from oracle import regrid as RG
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from cases import rough_case
from oracle.parity import oracle_bars

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def field_errors(got, exp):
    scale = np.abs(exp).max(axis=(1, 2))
    return np.abs(got - exp).max(axis=(1, 2)) / np.where(scale > 0, scale, 1.0)


def test_single_grid_sponge_fp64_parity():
    w = rough_case(73, 41, (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), seed=7)
    widths, rate = (1.2, 0.9, 0.0, 1.5), 4.0
    print("case", w.name, "sponge", widths, rate, flush=True)
    ctx = H.from_workloads([w])
    ctx.set_sponge(0, widths, rate)
    ctx.advance(w.dt, 15)
    r = O.from_workload(w)
    r.set_sponge(widths, rate)
    r.advance(w.dt, 15)
    err = field_errors(ctx.get_state(0), r.get_state())
    print("field errors", np.array2string(err, precision=2))
    assert np.all(err <= TOL)
    assert np.array_equal(ctx.get_mask(0), r.get_mask())
    ctx.close()


def test_patch_set_sponge_fp64_parity_and_mixed_gauges():
    w = W.amr_small(steps=3)
    L = 48 * w.dx0
    widths, rate = (0.3 * L, 0.0, 0.25 * L, 0.35 * L), 0.02
    gauges = {}
    for precision in (0, 1):
        print("case", w.name, "precision", precision, flush=True)
        ctx, ids = H.from_amr_workloads([w], precision=precision)
        ctx.set_sponge(0, widths, rate)
        ctx.advance(-1.0, 3)
        if precision == 0:
            runs = []

            def run(x):
                r = A.from_workload(x)
                r.set_sponge(widths, rate)
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
    ge = np.abs(gauges[1] - gauges[0]).max() / w.amplitude
    print("mixed vs FP64 gauge error / amplitude", ge)
    assert ge <= 1e-4


def test_regridded_patch_set_keeps_its_sponge():
    w = W.amr_small(steps=2)
    L = 48 * w.dx0
    widths, rate = (0.0, 0.3 * L, 0.3 * L, 0.0), 0.02
    ctx, ids = H.from_amr_workloads([w])
    ctx.set_sponge(0, widths, rate)
    ctx.advance(-1.0, 2)
    ctx.regrid(0, 0, tol=0.002, nbuf=2)
    ctx.advance(-1.0, 2)
    runs = []

    def run(x):
        r = A.from_workload(x)
        r.set_sponge(widths, rate)
        r.advance(x.dt, 2)
        r = RG.regrid(r, 0, tol=0.002, nbuf=2)
        r.set_sponge(widths, rate)
        r.advance(x.dt, 2)
        runs.append(r)
        return [r.get_state(k) for k in range(len(r.patches))]
    out, bars = oracle_bars(run, w)
    o = runs[0]
    assert len(ctx.patches()) == len(o.patches)
    for pid, p in enumerate(o.patches):
        err = field_errors(ctx.get_state(pid), out[pid])
        assert np.all(err <= bars[pid]), (pid, p.level, err, bars[pid])
    ctx.close()


def test_bad_sponges_are_refused():
    w = rough_case(41, 33, (W.BC_WALL,) * 4, seed=1)
    ctx = H.Context(w.params)
    ctx.add_grid(0, w.grid)
    with pytest.raises(H.HsgnError) as e:          # before finalize
        ctx.set_sponge(0, (1.0, 0.0, 0.0, 0.0), 1.0)
    assert e.value.code == H.HSGN_EINVAL
    ctx.finalize()
    for widths, rate, scen in (((-1.0, 0, 0, 0), 1.0, 0), ((1.0, 0, 0, 0), -1.0, 0),
                               ((float("nan"), 0, 0, 0), 1.0, 0), ((1.0, 0, 0, 0), float("inf"), 0),
                               ((1.0, 0, 0, 0), 1.0, 3)):
        with pytest.raises(H.HsgnError) as e:
            ctx.set_sponge(scen, widths, rate)
        assert e.value.code == H.HSGN_EINVAL
    ctx.close()


def test_split_step_with_a_sponge_is_bitwise_the_full_kernel(monkeypatch):
    """mixed precision with a sponge (the step-kernel instances compiled
    with it): the split step gives the bits of the full kernel, on an ocean
    with deep plain, shelf and dry coast and sponges on its open sides"""
    w = W.synthetic_ocean(n=512, dx=2000.0, steps=60)
    L = 512 * 2000.0
    runs = []
    for nosplit in ("0", "1"):
        monkeypatch.setenv("HSGN_NO_KERNEL_SPLIT", nosplit)
        print("case", w.name, "sponge, no_split", nosplit, flush=True)
        ctx = H.from_workloads([w], precision=1)
        ctx.set_sponge(0, (0.1 * L, 0.0, 0.08 * L, 0.08 * L), 0.01)
        ctx.advance(w.dt, 60)
        runs.append((ctx.get_state(0), ctx.get_mask(0), ctx.read_gauges(0)[1]))
        ctx.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
