"""GPU parity of the mbHSGN model (eq. mbHSGN) against the FP64 oracle.

Bar: FP64 fields within 1e-11 of the oracle, or, on the deep basin, within
ten times the oracle's own spread under one-ulp changes of the depths
(parity.py); masks equal, the sigma and p_b planes exactly zero; mixed
precision gauges within 1e-4 of the amplitude.
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def as_mb(w):
    w.params = W.Params(**{**w.params.__dict__, "model": 1})
    w.q[4] = 0.0
    w.q[6] = 0.0
    return w


def field_errors(got, exp):
    scale = np.abs(exp).max(axis=(1, 2))
    err = np.abs(got - exp).max(axis=(1, 2))
    return np.where(scale > 0, err / np.where(scale > 0, scale, 1.0), err)


@pytest.mark.parametrize("bc", [
    (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC),
    (W.BC_EXTRAP, W.BC_WALL, W.BC_EXTRAP, W.BC_WALL),
])
def test_rough_wet_dry_fp64_parity(bc):
    w = as_mb(rough_case(70, 45, bc, seed=5))
    print("case", w.name, "mbHSGN", flush=True)
    ctx = H.from_workloads([w])
    ctx.advance(0.0, 30)
    r = O.from_workload(w)
    r.advance(0.0, 30)
    got, exp = ctx.get_state(0), r.get_state()
    e = field_errors(got, exp)
    assert np.all(e <= TOL), e
    assert np.abs(got[4]).max() == 0.0 and np.abs(got[6]).max() == 0.0
    assert np.array_equal(ctx.get_mask(0), r.get_mask())
    assert ctx.clock(0)[2] == r.clock()[2]
    ctx.close()


def test_beach_reduced_fp64_parity():
    w = as_mb(W.beach_soliton(n=256, dx=0.2, steps=300))
    print("case", w.name, "mbHSGN", flush=True)
    ctx = H.from_workloads([w])
    ctx.advance(0.0, w.steps)
    r = O.from_workload(w)
    r.advance(0.0, w.steps)
    e = field_errors(ctx.get_state(0), r.get_state())
    assert np.all(e <= TOL), e
    _, eg = ctx.read_gauges(0)
    _, eo = r.read_gauges()
    assert np.abs(eg - eo).max() <= TOL * w.amplitude
    ctx.close()


def test_mixed_precision_gauges():
    w = as_mb(W.synthetic_ocean(n=512, dx=2000.0, steps=200))
    ctx = H.Context(w.params, precision=1)
    ctx.add_grid(0, w.grid)
    ctx.finalize()
    ctx.set_bathymetry(0, w.b)
    ctx.set_state(0, w.q)
    ctx.set_gauges(0, w.gauges)
    ctx.advance(w.dt, w.steps)
    r = O.from_workload(w)
    r.advance(w.dt, w.steps)
    _, eg = ctx.read_gauges(0)
    _, eo = r.read_gauges()
    err = np.abs(eg - eo).max() / w.amplitude
    print("mbHSGN mixed gauge error / amplitude", err)
    assert err <= 1e-4
    ctx.close()


def test_patch_set_fp64_parity():
    w = W.amr_small(steps=3)
    w.params = W.Params(**{**w.params.__dict__, "model": 1})
    ctx, ids = H.from_amr_workloads([w])
    ctx.advance(-1.0, w.steps)

    def run(x):
        o = A.from_workload(x)
        o.advance(x.dt, x.steps)
        return [o.get_state(k) for k in range(len(x.patches))]
    exp, bars = oracle_bars(run, w)
    for pid, k in zip(ids[0], range(len(w.patches))):
        e = field_errors(ctx.get_state(pid), exp[k])
        assert np.all(e <= bars[k]), (k, e, bars[k])
    ctx.close()
