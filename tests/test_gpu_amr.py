"""GPU parity of static patch sets (AMR) against the FP64 oracle.

Bar (FP64): every field of every patch within 1e-11 of the oracle relative
to that field's largest magnitude on the patch, or, on the deep basin, within
ten times the oracle's own spread under one-ulp changes of the depths
(parity.py); masks equal, gauges within 1e-11 of the amplitude.  The two
sides evaluate the method in independent operation orders.  Mixed
precision: gauges within 1e-4 of the amplitude.  The level-0 step of a patch set is replayed from a HIP
graph; the runs below replay it several times with host reads in between
and compare every intermediate state.
"""
import dataclasses

import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from cases import rough_case
from oracle.parity import TOL, field_errors, oracle_bars

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def amr_states(w, chunks):
    """oracle states of every patch after each chunk of level-0 steps"""
    o = A.from_workload(w)
    out = []
    for c in chunks:
        o.advance(w.dt, c)
        out += [o.get_state(k) for k in range(len(w.patches))]
    return out


def compare(ctx, ids, o, w, what, bars):
    worst = 0.0
    for pid, k in zip(ids, range(len(w.patches))):
        e = field_errors(ctx.get_state(pid), o.get_state(k))
        assert np.all(e <= bars[k]), "%s patch %d (level %d): %s bars %s" % (
            what, k, w.patches[k].level, np.array2string(e, precision=2),
            np.array2string(bars[k], precision=2))
        assert np.array_equal(ctx.get_mask(pid), o.get_mask(k)), (what, k)
        worst = max(worst, float(e.max()))
    return worst


def test_level0_tiling_matches_oracle_single_grid():
    bc = (W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC)
    w = rough_case(61, 47, bc, seed=5)
    t = W.tiled(w, 3, 2)
    print("case", t.name, flush=True)
    ctx, ids = H.from_amr_workloads([t])
    ctx.advance(-1.0, 12)
    ref = O.from_workload(w)
    ref.advance(w.dt, 12)
    q, m = ref.get_state(), ref.get_mask()
    for pid, p in zip(ids[0], t.patches):
        i0, j0 = int(round(p.x0 / w.grid.dx)), int(round(p.y0 / w.grid.dy))
        sl = (slice(j0, j0 + p.ny), slice(i0, i0 + p.nx))
        e = field_errors(ctx.get_state(pid), q[(slice(None),) + sl])
        assert np.all(e <= TOL), e
        assert np.array_equal(ctx.get_mask(pid), m[sl])
    ctx.close()


def test_three_levels_fp64_parity_across_graph_replays():
    w = W.amr_small(steps=6)
    print("case", w.name, flush=True)
    ctx, ids = H.from_amr_workloads([w])
    _, bars = oracle_bars(lambda x: amr_states(x, (1, 2, 3)), w)
    npch = len(w.patches)
    o = A.from_workload(w)
    worst = 0.0
    for c, chunk in enumerate((1, 2, 3)):      # graph replays with host reads between
        ctx.advance(-1.0, chunk)
        o.advance(w.dt, chunk)
        worst = max(worst, compare(ctx, ids[0], o, w, "after %d more steps" % chunk,
                                   bars[c * npch:(c + 1) * npch]))
        t, dtn, steps = ctx.clock(0)
        assert abs(t - o.t) <= 1e-12 * o.t and steps == o.steps
    print("worst relative field error", worst)
    tg, eg = ctx.read_gauges(0)
    to, eo = o.read_gauges()
    np.testing.assert_allclose(tg, to, rtol=1e-12)
    assert np.abs(eg - eo).max() <= TOL * w.amplitude
    d = ctx.diagnostics(0)
    assert abs(d["mass"] - o.mass()) <= 1e-13 * o.mass()
    assert d["steps"] == 6
    ctx.close()


def test_direct_launches_equal_graph_replays_bitwise():
    w = W.amr_small(steps=3)
    runs = []
    for timing in (False, True):
        ctx, ids = H.from_amr_workloads([w])
        ctx.set_timing(timing)
        ctx.advance(-1.0, w.steps)
        runs.append([ctx.get_state(pid) for pid in ids[0]])
        ctx.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_lake_at_rest_exact_fp64_and_mixed():
    w = W.amr_small(amp=0.0, steps=3)
    o = A.from_workload(w)
    o.prepare()
    for precision in (0, 1):
        ctx, ids = H.from_amr_workloads([w], precision=precision)
        for pid, p in zip(ids[0], o.patches):
            # at rest on the bathymetry as stored: FP32 in mixed precision
            # (the averaged-down coarse bathymetry rounded once)
            b = p.b[2:-2, 2:-2]
            if precision == 1:
                b = b.astype(np.float32).astype(np.float64)
            q = np.zeros((7, p.ny, p.nx))
            q[0] = np.maximum(-b, 0.0)
            ctx.set_state(pid, q)
        ctx.advance(-1.0, w.steps)
        for pid, p in zip(ids[0], o.patches):
            q = ctx.get_state(pid)
            assert np.abs(q[1:]).max() == 0.0, (precision, pid)
            if precision == 0:
                assert np.array_equal(q[0], np.maximum(-p.b[2:-2, 2:-2], 0.0))
        ctx.close()


def test_mass_conserved_on_device():
    w = W.amr_small(steps=6)
    ctx, ids = H.from_amr_workloads([w])
    ctx.advance(-1.0, 1)
    m1 = ctx.diagnostics(0)["mass"]
    ctx.advance(-1.0, 5)
    d = ctx.diagnostics(0)
    print("relative mass drift", (d["mass"] - m1) / m1)
    assert abs(d["mass"] - m1) <= 2e-15 * m1 and d["clipped_mass"] == 0.0
    ctx.close()


def test_mixed_gauges_within_1e4_of_amplitude():
    w = W.amr_small(steps=6)
    ctx, ids = H.from_amr_workloads([w], precision=1)
    ctx.advance(-1.0, w.steps)
    o = A.from_workload(w)
    o.advance(w.dt, w.steps)
    _, eg = ctx.read_gauges(0)
    _, eo = o.read_gauges()
    err = np.abs(eg - eo).max() / w.amplitude
    print("mixed gauge error / amplitude", err)
    assert err <= 1e-4
    ctx.close()


def test_patch_sets_and_single_grids_in_one_context():
    """an ensemble mixing a patch set and a single grid: each matches its
    own oracle run"""
    a = W.amr_small(steps=2)
    g = W.amr_small_uniform(0, steps=2)
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
    for pid, p in zip(ids, a.patches):
        ctx.set_state(pid, p.q)
    ctx.set_bathymetry(gid, g.b)
    ctx.set_state(gid, g.q)
    ctx.set_clock(0, 0.0, a.dt, 0)
    ctx.set_clock(1, 0.0, g.dt, 0)
    ctx.advance(-1.0, 2)
    _, bars = oracle_bars(lambda x: amr_states(x, (2,)), a)
    o = A.from_workload(a)
    o.advance(a.dt, 2)
    compare(ctx, ids, o, a, "patch set", bars)

    def grid_run(x):
        r = O.OracleGrid(x.params, x.grid)
        r.set_bathymetry(x.b)
        r.set_state(x.q)
        r.advance(x.dt, 2)
        return [r.get_state()]
    exp, gbar = oracle_bars(grid_run, g)
    e = field_errors(ctx.get_state(gid), exp[0])
    assert np.all(e <= gbar[0]), (e, gbar[0])
    ctx.close()


def test_adaptive_step_is_refused_for_patch_sets():
    w = W.amr_small(steps=1)
    ctx, ids = H.from_amr_workloads([w])
    assert ctx.advance_status(0.0, 1) == H.HSGN_ENOTSUP
    ctx.close()


def test_autotune_per_level_keeps_state_and_results():
    w = W.amr_small(steps=3)
    a, ids = H.from_amr_workloads([w])
    b, _ = H.from_amr_workloads([w])
    before = [b.get_state(pid) for pid in ids[0]]
    rows = b.autotune(trials=2)
    print("tile rows per level", rows, flush=True)
    assert len(rows) == 3
    for pid, q in zip(ids[0], before):
        assert np.array_equal(b.get_state(pid), q)
    a.advance(-1.0, w.steps)
    b.advance(-1.0, w.steps)
    for pid in ids[0]:
        assert np.array_equal(a.get_state(pid), b.get_state(pid))
    a.close()
    b.close()


def test_full_size_amr_ocean_properties():
    """the three-level AMR ocean of the benchmark at full size (2506 patches),
    with walls on the domain boundary so that no water leaves (the ring wave
    crosses the open boundary of the benchmark case, where the level-0 mass
    falls by 1.65e-10 of itself over these steps, as the oracle on level 0
    alone shows too): FP64 mass conserved over level-0 steps 2..4 to the
    rounding of the diagnostic itself, and the mixed form's gauges within
    1e-4 of the amplitude of the FP64 run.

    The diagnostic sums 256 patches of 128^2 cells: 16 cells per thread, a
    10-level tree, then the 256 patch sums in order on the host, so each
    evaluation carries at most about 280 ulps of relative rounding (3.1e-14);
    the bar on the difference of two evaluations is 1e-13."""
    w = dataclasses.replace(W.amr_ocean(), bc=(W.BC_WALL,) * 4)
    print("case", w.name, "walls", flush=True)
    gauges = {}
    for precision in (0, 1):
        ctx, ids = H.from_amr_workloads([w], precision=precision)
        ctx.advance(-1.0, 1)
        m1 = ctx.diagnostics(0)["mass"]
        c1 = ctx.diagnostics(0)["clipped_mass"]
        ctx.advance(-1.0, 3)
        d = ctx.diagnostics(0)
        drift = abs(d["mass"] - m1 - (d["clipped_mass"] - c1)) / m1
        print("precision", precision, "relative mass drift", drift, flush=True)
        assert drift <= (1e-13 if precision == 0 else 1e-6)
        gauges[precision] = ctx.read_gauges(0)[1]
        ctx.close()
    err = np.abs(gauges[1] - gauges[0]).max() / w.amplitude
    print("mixed vs FP64 gauge error / amplitude", err)
    assert err <= 1e-4


@pytest.mark.parametrize("mode", ["graph", "direct", "autotune"])
def test_split_patch_set_step_is_bitwise_the_full_kernel(monkeypatch, mode):
    """patch sets in mixed precision: the step split into patches' items
    away from the SWE region and the shore (kernel without the FP64 edge
    solve) and the rest (full kernel) gives the same bits as the full kernel
    on every item.  A small three-level ocean whose level 0 holds the shelf
    and the dry coast and whose finer levels lie in deep water; graph
    replays, direct launches (timing on) and after the autotuner"""
    w = W.amr_ocean(n=512, tile=64, targets=(40, 50), steps=4)
    runs = []
    for nosplit in ("0", "1"):
        monkeypatch.setenv("HSGN_NO_KERNEL_SPLIT", nosplit)
        print("case", w.name, mode, "no_split", nosplit, flush=True)
        ctx, ids = H.from_amr_workloads([w], precision=1)
        if mode == "direct":
            ctx.set_timing(True)
        if mode == "autotune":
            ctx.autotune(trials=1)
        ctx.advance(-1.0, 4)
        runs.append(([(ctx.get_state(p), ctx.get_mask(p)) for p in ids[0]], ctx.read_gauges(0)[1]))
        ctx.close()
    (a, ga), (b, gb) = runs
    assert np.array_equal(ga, gb)
    for k, ((qa, ma), (qb, mb)) in enumerate(zip(a, b)):
        assert np.array_equal(qa, qb) and np.array_equal(ma, mb), k


@pytest.mark.parametrize("mapped", [False, True])
def test_packed_strips_give_the_unpacked_state_bitwise(monkeypatch, mapped):
    """narrow strips of patch-set patches packed into shared wavefronts (the
    default) against one wavefront per strip (HSGN_NO_PACKING=1): fewer work
    items, the same state bit for bit in both precisions (the clipped mass,
    summed per item, may round differently).  Mapped patch sets in mixed
    precision are not packed: the same work items."""
    from test_oracle_amr_mapped import L48, bumpy, with_momentum
    w = with_momentum(W.amr_small(steps=3))
    nodes = None
    if mapped:
        w = dataclasses.replace(w, dt=0.7 * w.dt)
        nodes = [W.nested_nodes(w, bumpy(L48, L48))]
    for precision in (0, 1):
        print("case packing, mapped", mapped, "precision", precision, flush=True)
        runs = []
        for nopack in ("0", "1"):
            monkeypatch.setenv("HSGN_NO_PACKING", nopack)
            ctx, ids = H.from_amr_workloads([w], precision=precision, nodes=nodes)
            n = ctx.work_items()
            ctx.advance(-1.0, w.steps)
            runs.append((n, [ctx.get_state(pid) for pid in ids[0]],
                         [ctx.get_mask(pid) for pid in ids[0]]))
            ctx.close()
        if mapped and precision == 1:
            assert runs[0][0] == runs[1][0], (runs[0][0], runs[1][0])
        else:
            assert runs[0][0] < runs[1][0], (runs[0][0], runs[1][0])
        for k, (a, b) in enumerate(zip(runs[0][1], runs[1][1])):
            assert np.array_equal(a, b), (precision, k)
        for a, b in zip(runs[0][2], runs[1][2]):
            assert np.array_equal(a, b)
