"""The radially symmetric hump (Sec. 5, radially symmetric tests) on a
three-level patch set on the GPU, against the radial 1D reference of
Appendix D computed by the oracle (x the radius, the geometric source
terms; pinned in test_oracle_radial.py).

The hump (H = 100 m, A = 5 m, sigma = 100 m, alpha = 3) sits at the centre
of the domain; level 1 covers 800 m and level 2 200 m around it (ratios 4,
4), at level-0 spacings of 50 m and 25 m.  Bar: along the diagonal, at
t = 6 s, the finest level's surface is within 2e-3 of the amplitude of the
radial solution, far closer than level 0 alone (at most 5% of its error),
and the error falls when level 0 is refined.
"""
import numpy as np
import pytest

from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from test_oracle_radial import finest_diagonal, radial_profile

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEPTH = W.RADIAL["H"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def test_three_level_radial_hump_against_the_radial_reference():
    rr, ref = radial_profile(0.5, rmax=2000.0)
    errs = []
    for n0, dx0 in ((48, 50.0), (96, 25.0)):
        w = W.radial_hump_amr(n0, dx0)
        ctr = 0.5 * n0 * dx0
        print("case", w.name, w.steps, "level-0 steps", flush=True)
        ctx, ids = H.from_amr_workloads([w])
        ctx.advance(-1.0, w.steps)
        pts = finest_diagonal(w, [ctx.get_state(pid) for pid in ids[0]], ctr)
        ctx.close()
        err = np.abs(pts[:, 1] - np.interp(pts[:, 0], rr, ref)).max()
        p0 = w.patches[0]
        g = W.Workload("level0", w.params, W.Grid(n0, n0, 0.0, 0.0, dx0, dx0, w.bc), p0.b, p0.q,
                       np.zeros((0, 2)), w.steps, w.dt, w.amplitude)
        c0 = H.from_workloads([g], gauges=False)
        c0.advance(w.dt, w.steps)
        q0 = c0.get_state(0)
        c0.close()
        x = (np.arange(n0) + 0.5) * dx0
        err0 = np.abs(np.array([q0[0, i, i] for i in range(n0)]) - DEPTH
                      - np.interp(np.sqrt(2.0) * np.abs(x - ctr), rr, ref)).max()
        print("  three levels %.3e, level 0 alone %.3e" % (err, err0), flush=True)
        assert set(pts[:, 2].astype(int)) == {0, 1, 2}
        assert err < 0.05 * err0 and err < 2e-3 * W.RADIAL["A"]
        errs.append(err)
    assert errs[1] < errs[0]
