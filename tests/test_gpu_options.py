"""GPU parity for every run option of the step (FP64, bar 1e-11).

The rough wet/dry case (ragged tiles, two boundary conditions, SWE and
dispersive cells, breaking) is advanced with each limiter, without the
transverse waves, with Lie splitting, with every cell in the SWE region,
with the widest and the narrowest transition neighbourhood, with a fixed
relaxation parameter and for mbHSGN with the first-order limiter, and
compared with the oracle run with the same option.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from cases import rough_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11

OPTIONS = {
    "first_order": dict(limiter=0),
    "minmod": dict(limiter=1),
    "unlimited": dict(limiter=3),
    "no_transverse": dict(transverse=0),
    "lie": dict(splitting=0),
    "all_swe": dict(h_star=1e6),
    "neighbourhood_0": dict(nbr_n=0),
    "neighbourhood_2": dict(nbr_n=2),
    "fixed_c2": dict(c2=40.0),
    "mbhsgn_first_order": dict(model=1, limiter=0),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


@pytest.mark.parametrize("name", sorted(OPTIONS))
def test_option_fp64_parity(name):
    w = rough_case(73, 41, (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), seed=11)
    w.params = dataclasses.replace(w.params, **OPTIONS[name])
    if w.params.model == 1:
        w.q[4] = 0.0
        w.q[6] = 0.0
    print("case", w.name, name, flush=True)
    ctx = H.from_workloads([w])
    ctx.advance(w.dt, 15)
    r = O.from_workload(w)
    r.advance(w.dt, 15)
    got, exp = ctx.get_state(0), r.get_state()
    scale = np.abs(exp).max(axis=(1, 2))
    err = np.abs(got - exp).max(axis=(1, 2)) / np.where(scale > 0, scale, 1.0)
    print("field errors", np.array2string(err, precision=2))
    assert np.all(err <= TOL)
    assert np.array_equal(ctx.get_mask(0), r.get_mask())
    tg, eg = ctx.read_gauges(0)
    to, eo = r.read_gauges()
    assert np.abs(eg - eo).max() <= TOL * w.amplitude
    ctx.close()
