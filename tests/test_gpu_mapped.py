"""GPU parity of mapped grids (Sec. 4, mapped grids; FP64 single grids)
through the C ABI.

Bar: fields within 1e-11 of the oracle relative to each field's largest
magnitude (the two sides evaluate the method in independent operation
orders), masks equal; on the GPU the identity mapping of a Cartesian grid
gives the Cartesian kernel's results, and a Cartesian scenario stepped in the
same launch as a mapped one (by the mapped kernel) the results it has alone,
both to the same bar (the two kernels fuse products into sums differently,
so their bits differ); capacity-weighted mass against the oracle's;
in mixed precision the gauges within 1e-4 of the amplitude of the FP64
mapped run and a lake at rest exact; unsupported combinations refused.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from cases import rough_case
from test_oracle_mapped import BCS, distorted, dyadic_case, nodes, periodic_case

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


def gpu_run(w, xy, steps, dt):
    ctx = H.from_workloads([w])
    if xy is not None:
        ctx.set_mapping(0, *xy)
    ctx.advance(dt, steps)
    out = ctx.get_state(0), ctx.get_mask(0), ctx.diagnostics(0)
    ctx.close()
    return out


def oracle_run(w, xy, steps, dt):
    r = O.from_workload(w)
    if xy is not None:
        r.set_mapping(*xy)
    r.advance(dt, steps)
    return r.get_state(), r.get_mask(), r.mass()


@pytest.mark.parametrize("bc", BCS)
def test_identity_mapping_gives_the_cartesian_results(bc):
    w = dyadic_case(bc, seed=21)
    print("case", w.name, "identity mapping", flush=True)
    xy = nodes(w.grid, lambda x, y: x, lambda x, y: y)
    qm, mm, _ = gpu_run(w, xy, 12, w.dt)
    qc, mc, _ = gpu_run(w, None, 12, w.dt)
    qo, mo, _ = oracle_run(w, None, 12, w.dt)
    print("identity mapping vs Cartesian kernel", np.array2string(field_errors(qm, qc), precision=2))
    assert np.all(field_errors(qm, qc) <= TOL)
    assert np.array_equal(mm, mc)
    assert np.all(field_errors(qm, qo) <= TOL)
    assert np.array_equal(mm, mo)


def mapped_cases():
    rot = rough_case(40, 36, (W.BC_WALL, W.BC_WALL, W.BC_PERIODIC, W.BC_PERIODIC), seed=22)
    rot = dataclasses.replace(rot, gauges=np.zeros((0, 2)))
    c, s = np.cos(0.6), np.sin(0.6)
    yield "rotated_walls", rot, rot.dt, nodes(rot.grid, lambda x, y: c * x - s * y, lambda x, y: s * x + c * y)
    scl = dyadic_case(BCS[1], seed=23)
    yield "scaled_walls", scl, 0.5 * scl.dt, nodes(scl.grid, lambda x, y: 2.0 * x, lambda x, y: 0.5 * y)
    dis = rough_case(61, 47, (W.BC_WALL, W.BC_EXTRAP, W.BC_WALL, W.BC_EXTRAP), seed=24)
    dis = dataclasses.replace(dis, gauges=np.zeros((0, 2)))
    yield "distorted_walls_wetdry", dis, 0.8 * dis.dt, distorted(dis.grid, amp=0.02)


@pytest.mark.parametrize("name", ["rotated_walls", "scaled_walls", "distorted_walls_wetdry"])
def test_mapped_grid_fp64_parity(name):
    w, dt, xy = next((w, dt, xy) for n, w, dt, xy in mapped_cases() if n == name)
    print("case", name, w.name, flush=True)
    qg, mg, _ = gpu_run(w, xy, 12, dt)
    qo, mo, _ = oracle_run(w, xy, 12, dt)
    err = field_errors(qg, qo)
    print("field errors", np.array2string(err, precision=2), "bitwise", np.array_equal(qg, qo))
    assert np.all(err <= TOL)
    assert np.array_equal(mg, mo)


def test_distorted_periodic_hump_parity_and_mass():
    nx, ny = 64, 48
    g = periodic_case(np.zeros((7, ny, nx)), np.zeros((ny, nx)), nx=nx, ny=ny).grid
    X, Y = W.cell_centres(g)
    q = np.zeros((7, ny, nx))
    q[0] = 1.0 + 0.1 * np.exp(-((X - 6.0) ** 2 + (Y - 6.0) ** 2))
    q[1] = 0.05 * q[0]
    w = periodic_case(q, np.full((ny, nx), -1.0), nx=nx, ny=ny)
    xy = distorted(g)
    print("case distorted periodic hump", flush=True)
    qg, _, dg = gpu_run(w, xy, 30, w.dt)
    qo, _, mo = oracle_run(w, xy, 30, w.dt)
    err = field_errors(qg, qo)
    print("field errors", np.array2string(err, precision=2))
    assert np.all(err <= TOL)
    assert abs(dg["mass"] - mo) <= 1e-13 * mo


def test_cartesian_scenario_beside_a_mapped_one_keeps_its_results():
    a = dyadic_case(BCS[0], seed=25)
    b = rough_case(40, 36, (W.BC_WALL, W.BC_WALL, W.BC_PERIODIC, W.BC_PERIODIC), seed=26)
    b = dataclasses.replace(b, gauges=np.zeros((0, 2)), dt=a.dt)
    c, s = np.cos(0.3), np.sin(0.3)
    xy = nodes(b.grid, lambda x, y: c * x - s * y, lambda x, y: s * x + c * y)
    print("case ensemble: Cartesian", a.name, "+ rotated", b.name, flush=True)
    ctx = H.from_workloads([a, b])
    ctx.set_mapping(1, *xy)
    ctx.advance(a.dt, 10)
    qa, qb = ctx.get_state(0), ctx.get_state(1)
    ctx.close()
    assert np.all(field_errors(qa, gpu_run(a, None, 10, a.dt)[0]) <= TOL)
    assert np.all(field_errors(qa, oracle_run(a, None, 10, a.dt)[0]) <= TOL)
    assert np.all(field_errors(qb, oracle_run(b, xy, 10, a.dt)[0]) <= TOL)


def test_unsupported_mappings_are_refused():
    w = dyadic_case(BCS[0], seed=27)
    xy = nodes(w.grid, lambda x, y: x, lambda x, y: y)
    ctx = H.from_workloads([w])
    with pytest.raises(H.HsgnError) as e:
        ctx.set_mapping(0, -xy[0], xy[1])            # clockwise cells
    assert e.value.code == H.HSGN_EINVAL
    ctx.set_sponge(0, (0.5, 0.0, 0.0, 0.0), 1.0)
    with pytest.raises(H.HsgnError) as e:
        ctx.set_mapping(0, *xy)
    assert e.value.code == H.HSGN_ENOTSUP
    ctx.close()
    ctx = H.from_workloads([w])
    ctx.set_mapping(0, *xy)
    with pytest.raises(H.HsgnError) as e:
        ctx.set_sponge(0, (0.5, 0.0, 0.0, 0.0), 1.0)
    assert e.value.code == H.HSGN_ENOTSUP
    ctx.close()


def test_mixed_precision_mapped_gauges_against_fp64():
    w = rough_case(61, 47, (W.BC_WALL, W.BC_EXTRAP, W.BC_WALL, W.BC_EXTRAP), seed=28)
    xy = distorted(w.grid, amp=0.02)
    dt = 0.8 * w.dt
    rec = {}
    for precision in (0, 1):
        print("case", w.name, "distorted, precision", precision, flush=True)
        ctx = H.from_workloads([w], precision=precision)
        ctx.set_mapping(0, *xy)
        ctx.advance(dt, 30)
        rec[precision] = ctx.read_gauges(0)[1]
        ctx.close()
    ge = np.abs(rec[1] - rec[0]).max() / w.amplitude
    print("mixed vs FP64 gauge error / amplitude", ge)
    assert rec[0].shape == rec[1].shape and rec[0].size > 0
    assert ge <= 1e-4


def test_mixed_precision_lake_at_rest_on_a_distorted_grid_is_exact():
    nx, ny = 40, 32
    rng = np.random.default_rng(29)
    b = W.fp32_representable(-1.0 - 0.3 * rng.random((ny, nx)))
    q = np.zeros((7, ny, nx))
    q[0] = -b
    w = periodic_case(q, b)
    print("case mixed lake at rest, distorted", flush=True)
    ctx = H.from_workloads([w], precision=1)
    ctx.set_mapping(0, *distorted(w.grid))
    ctx.advance(w.dt, 20)
    s = ctx.get_state(0)
    ctx.close()
    assert np.abs(s[0] + b).max() == 0.0
    assert np.abs(s[1:]).max() == 0.0


def test_mixed_mapped_split_step_is_bitwise_the_full_kernel(monkeypatch):
    """mixed precision on a mapped ocean with deep plain, shelf and dry coast:
    the split step (items without near-shore edges on the kernel compiled
    without the FP64 re-solve) gives the bits of the full kernel"""
    w = W.synthetic_ocean(n=512, dx=2000.0, steps=40)
    g = w.grid
    xi = g.x0 + np.arange(-2, g.nx + 3) * g.dx
    eta = g.y0 + np.arange(-2, g.ny + 3) * g.dy
    XI, ETA = np.meshgrid(xi, eta)
    L = g.nx * g.dx
    xy = (XI + 0.005 * L * np.sin(2 * np.pi * ETA / L), ETA + 0.005 * L * np.sin(2 * np.pi * XI / L))
    runs = []
    for nosplit in ("0", "1"):
        monkeypatch.setenv("HSGN_NO_KERNEL_SPLIT", nosplit)
        print("case", w.name, "mapped, no_split", nosplit, flush=True)
        ctx = H.from_workloads([w], precision=1)
        ctx.set_mapping(0, *xy)
        ctx.advance(0.85 * w.dt, 40)
        runs.append((ctx.get_state(0), ctx.get_mask(0), ctx.read_gauges(0)[1]))
        ctx.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_mapping_set_between_graph_replays_beside_a_patch_set():
    """a context with a patch set (its level-0 step replayed from a HIP
    graph) and a single grid of the same deep basin: after one step, the
    single grid is mapped (rotated); the next steps run the mapped kernel
    (the graph captured before holds the Cartesian one and is dropped), and
    a regrid is then refused because the rebuilt context would not carry
    the mapping.  Deep water: the FP64 bar of oracle/parity.py."""
    from oracle import amr as A
    from oracle.parity import oracle_bars
    a = W.amr_small(steps=3)
    g = dataclasses.replace(W.amr_small_uniform(0, steps=3), gauges=np.zeros((0, 2)))
    c, s = np.cos(0.4), np.sin(0.4)
    xy = nodes(g.grid, lambda x, y: c * x - s * y, lambda x, y: s * x + c * y)
    ctx = H.Context(a.params)
    ids = []
    for p in a.patches:
        d = 4.0 ** p.level
        grid = W.Grid(p.nx, p.ny, p.x0, p.y0, a.dx0 / d, a.dy0 / d, a.bc)
        ids.append(ctx.add_grid(0, grid, level=p.level))
    gid = ctx.add_grid(1, g.grid)
    ctx.finalize()
    for pid, p in zip(ids, a.patches):
        ctx.set_bathymetry(pid, p.b)
        ctx.set_state(pid, p.q)
    ctx.set_bathymetry(gid, g.b)
    ctx.set_state(gid, g.q)
    ctx.set_clock(0, 0.0, a.dt, 0)
    ctx.set_clock(1, 0.0, g.dt, 0)
    ctx.advance(-1.0, 1)
    ctx.set_mapping(gid, *xy)
    ctx.advance(-1.0, 2)

    def mapped_run(x, extra=0):
        r = O.from_workload(x)
        r.advance(x.dt, 1)
        r.set_mapping(*xy)
        r.advance(x.dt, 2 + extra)
        return [r.get_state()]
    exp, gbar = oracle_bars(mapped_run, g)
    err = field_errors(ctx.get_state(gid), exp[0])
    print("mapped grid beside a patch set", np.array2string(err, precision=2),
          "bars", np.array2string(gbar[0], precision=2), flush=True)
    assert np.all(err <= gbar[0])

    def run(x):
        o = A.from_workload(x)
        o.advance(x.dt, 3)
        return [o.get_state(k) for k in range(len(x.patches))]
    exp, bars = oracle_bars(run, a)
    for pid, k in zip(ids, range(len(a.patches))):
        assert np.all(field_errors(ctx.get_state(pid), exp[k]) <= bars[k]), k
    with pytest.raises(H.HsgnError) as e:
        ctx.regrid(0, 0, tol=0.002)
    assert e.value.code == H.HSGN_ENOTSUP
    ctx.advance(-1.0, 1)                       # still usable, still mapped
    exp, gbar = oracle_bars(lambda x: mapped_run(x, 1), g)
    assert np.all(field_errors(ctx.get_state(gid), exp[0]) <= gbar[0])
    ctx.close()
