"""Full-size FP64 parity: the 1024^2 plane beach (wet/dry fronts, breaking
latch, walls, 16 gauges) at its full size, in the launch configuration the
benchmark times, against the FP64 oracle over 200 adaptive steps.

Bar (shallow water, depth 1 m): every field within 1e-11 of the oracle
relative to its largest magnitude, masks equal, the same step count, clocks
to 1e-12, gauges within 1e-11 of the amplitude.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.parity import TOL, field_errors
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def test_beach_1024_full_size_200_steps():
    w = W.beach_soliton(steps=200)
    print("case", w.name, w.steps, "adaptive steps", flush=True)
    ctx = H.from_workloads([w])
    ctx.autotune()                       # the benchmark's launch configuration
    ctx.advance(0.0, w.steps)
    r = O.from_workload(w)
    r.advance(0.0, w.steps)
    e = field_errors(ctx.get_state(0), r.get_state())
    print("field errors", np.array2string(e, precision=2), flush=True)
    assert np.all(e <= TOL)
    assert np.array_equal(ctx.get_mask(0), r.get_mask())
    t, _, steps = ctx.clock(0)
    rt, _, rsteps, _ = r.clock()
    assert steps == rsteps == w.steps
    assert abs(t - rt) <= 1e-12 * rt
    tg, eg = ctx.read_gauges(0)
    to, eo = r.read_gauges()
    np.testing.assert_allclose(tg, to, rtol=1e-12)
    assert np.abs(eg - eo).max() <= TOL * w.amplitude
    ctx.close()
