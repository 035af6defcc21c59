"""GPU parity of mapped patch sets (Sec. 4, mapped grids, on static patch
sets) against the FP64 oracle, through the C ABI.

Bar (FP64): the patch-set bar of oracle/parity.py: every field of every
patch within max(1e-11, 10 x the oracle's own spread under one-ulp changes
of the depths), relative to the field's largest magnitude on the patch;
masks equal; gauges within 1e-11 of the amplitude; the capacity-weighted
mass within 1e-13 of the oracle's.  On wet/dry data in shallow water the bar
is 1e-11 itself.  Mixed precision: gauges within 1e-4 of the amplitude.  The
level-0 step is replayed from a HIP graph with host reads between replays.
"""
import dataclasses

import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from oracle.parity import TOL, field_errors, oracle_bars
from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

from cases import rough_case
from test_oracle_amr_mapped import L48, bumpy, identity, periodic_bumpy, turned, with_momentum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    H.lib()
    yield


def basin(steps, fmap, bc=(W.BC_WALL,) * 4, amp=1.0, momentum=True):
    """the three-level basin at 0.7 of its step (the distorted cells are
    smaller), its nodes under fmap"""
    w = W.amr_small(steps=steps, bc=bc, amp=amp)
    if momentum:
        w = with_momentum(w)
    w = dataclasses.replace(w, dt=0.7 * w.dt)
    return w, W.nested_nodes(w, fmap)


def oracle_states(w, nodes, chunks):
    o = A.from_workload(w, nodes=nodes)
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


def test_distorted_three_levels_fp64_parity_across_graph_replays():
    w, nodes = basin(3, bumpy(L48, L48))
    print("case distorted three-level basin, walls, 1 + 2 steps", flush=True)
    ctx, ids = H.from_amr_workloads([w], nodes=[nodes])
    _, bars = oracle_bars(lambda x: oracle_states(x, nodes, (1, 2)), w)
    npch = len(w.patches)
    o = A.from_workload(w, nodes=nodes)
    worst = 0.0
    for c, chunk in enumerate((1, 2)):
        ctx.advance(-1.0, chunk)
        o.advance(w.dt, chunk)
        worst = max(worst, compare(ctx, ids[0], o, w, "after %d more steps" % chunk,
                                   bars[c * npch:(c + 1) * npch]))
        t, _, steps = ctx.clock(0)
        assert abs(t - o.t) <= 1e-12 * o.t and steps == o.steps
    print("worst relative field error", worst)
    tg, eg = ctx.read_gauges(0)
    to, eo = o.read_gauges()
    np.testing.assert_allclose(tg, to, rtol=1e-12)
    assert np.abs(eg - eo).max() <= TOL * w.amplitude
    d = ctx.diagnostics(0)
    assert abs(d["mass"] - o.mass()) <= 1e-13 * o.mass()
    ctx.close()


def test_direct_launches_equal_graph_replays_bitwise():
    w, nodes = basin(2, turned(bumpy(L48, L48), 0.5))
    print("case rotated distorted basin, graph against direct launches", flush=True)
    runs = []
    for timing in (False, True):
        ctx, ids = H.from_amr_workloads([w], nodes=[nodes])
        ctx.set_timing(timing)
        ctx.advance(-1.0, w.steps)
        runs.append([ctx.get_state(pid) for pid in ids[0]])
        ctx.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("bc, tiles", [
    ((W.BC_WALL, W.BC_EXTRAP, W.BC_PERIODIC, W.BC_PERIODIC), (3, 2)),
    ((W.BC_WALL, W.BC_WALL, W.BC_WALL, W.BC_EXTRAP), (2, 3)),
])
def test_level0_tiling_of_a_rotated_distorted_wet_dry_grid(bc, tiles):
    w = rough_case(61, 47, bc, seed=5)
    g = w.grid
    w = dataclasses.replace(w, dt=0.8 * w.dt)
    fmap = turned(bumpy(g.nx * g.dx, g.ny * g.dy, amp=0.02), 0.6)
    t = W.tiled(w, *tiles)
    print("case", t.name, "rotated, distorted", flush=True)
    ctx, ids = H.from_amr_workloads([t], nodes=[W.nested_nodes(t, fmap)])
    ctx.advance(-1.0, 12)
    ref = O.from_workload(w)
    XI, ETA = np.meshgrid(g.x0 + np.arange(-2, g.nx + 3) * g.dx, g.y0 + np.arange(-2, g.ny + 3) * g.dy)
    ref.set_mapping(*fmap(XI, ETA))
    ref.advance(w.dt, 12)
    q, m = ref.get_state(), ref.get_mask()
    worst = 0.0
    for pid, p in zip(ids[0], t.patches):
        i0, j0 = int(round(p.x0 / g.dx)), int(round(p.y0 / g.dy))
        sl = (slice(j0, j0 + p.ny), slice(i0, i0 + p.nx))
        e = field_errors(ctx.get_state(pid), q[(slice(None),) + sl])
        assert np.all(e <= TOL), (pid, e)
        assert np.array_equal(ctx.get_mask(pid), m[sl]), pid
        worst = max(worst, float(e.max()))
    print("worst relative field error", worst)
    ctx.close()


def test_capacity_weighted_mass_conserved_on_device():
    w, nodes = basin(6, periodic_bumpy(L48, L48), bc=(W.BC_PERIODIC,) * 4)
    print("case periodic distorted basin, mass", flush=True)
    ctx, ids = H.from_amr_workloads([w], nodes=[nodes])
    ctx.advance(-1.0, 1)
    m1 = ctx.diagnostics(0)["mass"]
    ctx.advance(-1.0, 5)
    d = ctx.diagnostics(0)
    drift = abs(d["mass"] - m1) / m1
    o = A.from_workload(w, nodes=nodes)
    o.advance(w.dt, 6)
    print("relative mass drift %.2e, against the oracle %.2e" % (drift, abs(d["mass"] - o.mass()) / o.mass()))
    assert drift <= 1e-14 and d["clipped_mass"] == 0.0
    assert abs(d["mass"] - o.mass()) <= 1e-13 * o.mass()
    ctx.close()


def test_lake_at_rest_exact_fp64_and_mixed():
    w, nodes = basin(3, bumpy(L48, L48), amp=0.0, momentum=False)
    o = A.from_workload(w, nodes=nodes)
    o.prepare()
    for precision in (0, 1):
        print("case distorted lake at rest, precision", precision, flush=True)
        ctx, ids = H.from_amr_workloads([w], precision=precision, nodes=[nodes])
        for pid, p in zip(ids[0], o.patches):
            # at rest on the capacity-weighted bathymetry as stored (FP32 in
            # mixed precision: the averaged-down coarse bathymetry rounded once)
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
                assert np.array_equal(q[0], np.maximum(-p.b[2:-2, 2:-2], 0.0)), pid
        ctx.close()


def test_mixed_gauges_within_1e4_of_amplitude():
    w, nodes = basin(6, bumpy(L48, L48))
    print("case distorted basin, mixed precision", flush=True)
    ctx, ids = H.from_amr_workloads([w], precision=1, nodes=[nodes])
    ctx.advance(-1.0, w.steps)
    o = A.from_workload(w, nodes=nodes)
    o.advance(w.dt, w.steps)
    _, eg = ctx.read_gauges(0)
    _, eo = o.read_gauges()
    err = np.abs(eg - eo).max() / w.amplitude
    print("mixed gauge error / amplitude", err)
    assert err <= 1e-4
    ctx.close()


def test_mapped_and_cartesian_patch_sets_in_one_context():
    """two patch sets in one context, the first mapped (identity nodes: the
    Cartesian patch set's own oracle results) and the second distorted; the
    mapped kernel steps both, each to its own oracle run"""
    a = with_momentum(W.amr_small(steps=2))
    b, nb = basin(2, bumpy(L48, L48))
    a = dataclasses.replace(a, dt=b.dt)
    na = W.nested_nodes(a, identity)
    print("case identity-mapped and distorted patch sets together", flush=True)
    ctx, ids = H.from_amr_workloads([a, b], nodes=[na, nb])
    ctx.advance(-1.0, 2)
    for w, nodes, pids in ((a, None, ids[0]), (b, nb, ids[1])):
        _, bars = oracle_bars(lambda x: oracle_states(x, nodes, (2,)), w)
        o = A.from_workload(w, nodes=nodes)
        o.advance(w.dt, 2)
        compare(ctx, pids, o, w, "patch set", bars)
    ctx.close()


def test_patch_set_mapped_in_part_is_refused():
    w, nodes = basin(1, identity, momentum=False)
    print("case patch set mapped in part", flush=True)
    ctx, ids = H.from_amr_workloads([w])
    ctx.set_mapping(ids[0][0], *nodes[0])
    with pytest.raises(H.HsgnError) as e:
        ctx.advance(-1.0, 1)
    assert e.value.code == H.HSGN_EINVAL
    for pid, xy in zip(ids[0][1:], nodes[1:]):
        ctx.set_mapping(pid, *xy)
    ctx.advance(-1.0, 1)              # complete now
    ctx.close()
