"""Full-size and full-horizon FP64 parity on the GPU, too long for the test
suite (minutes of oracle time on the host); run on a GPU machine as

    python tests/fullsize_checks.py --case c5link [--steps 3000] [--out FILE]
    python tests/fullsize_checks.py --case c4step [--mapped] [--out FILE]

c5link: the smallest scenario of the 48-scenario ensemble (513^2 at its own
spacing) advanced over the ensemble's full 3000 fixed steps by the HIP path
(inside the 48-scenario FP64 launch of the benchmark) and by the oracle,
compared field by field, with the gauges.

c4step: the full three-level AMR ocean (256 level-0 patches of 128^2, 1000
level-1 and 1250 level-2 patches of 16..128 cells; 105.9 M cell updates)
advanced one level-0 step (with its 4 + 16 substeps) in FP64 by the HIP
path, in the launch configuration of the benchmark (autotuned tiles, the
step replayed from a HIP graph), and by the AMR oracle; every patch
compared.  Most patches lie where the wave has not yet arrived, so their
fields are round-off noise: errors there are taken relative to each field's
largest magnitude over the whole patch set, not over the patch.  With
--mapped the set lies on the smoothly distorted grid of
workloads.distorted_patch_nodes (nested nodes on every level) and steps at
0.85 of the Cartesian step, as in the benchmark's --mapped run.

Bar: the FP64 parity bar (oracle/parity.py): every field within
max(1e-11, 10 x the oracle's spread under one-ulp changes of the depths,
one twin run), masks equal, gauges within 1e-11 of the amplitude.  Prints
one JSON line with the errors, the bars and the timings.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import amr as A                                       # noqa: E402
from oracle import oracle as O                                    # noqa: E402
from oracle.parity import SPREAD, TOL, field_errors, oracle_bars, twin   # noqa: E402
from paper_2606_12162_amd import hsgn as H                        # noqa: E402
from paper_2606_12162_amd import workloads as W                   # noqa: E402


def c4step(args):
    w = W.amr_ocean()
    nodes = None
    if args.mapped:
        nodes = W.distorted_patch_nodes(w)
        w.dt = 0.85 * w.dt
    print("case", w.name, "mapped" if nodes else "", len(w.patches), "patches, one level-0 step",
          flush=True)
    t0 = time.perf_counter()
    ctx, ids = H.from_amr_workloads([w], precision=0, nodes=None if nodes is None else [nodes])
    ctx.autotune()
    ctx.advance(-1.0, 1)
    got = [ctx.get_state(pid) for pid in ids[0]]
    masks = [ctx.get_mask(pid) for pid in ids[0]]
    mass = ctx.diagnostics(0)["mass"]
    ctx.close()
    t_gpu = time.perf_counter() - t0
    print("GPU done in %.1f s" % t_gpu, flush=True)
    runs = []

    def run(x):
        o = A.from_workload(x, nodes=nodes)
        o.advance(x.dt, 1)
        runs.append(o)
        print("oracle run done", flush=True)
        return [o.get_state(k) for k in range(len(x.patches))]

    t1 = time.perf_counter()
    exp = run(w)
    twin_states = run(twin(w, 1))
    t_orc = time.perf_counter() - t1
    o = runs[0]
    scale = np.max([np.abs(e).max(axis=(1, 2)) for e in exp], axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    err = np.max([np.abs(g - e).max(axis=(1, 2)) for g, e in zip(got, exp)], axis=0) / scale
    spread = np.max([np.abs(t - e).max(axis=(1, 2)) for t, e in zip(twin_states, exp)],
                    axis=0) / scale
    bar = np.maximum(TOL, SPREAD * spread)
    masks_ok = all(np.array_equal(masks[k], o.get_mask(k)) for k in range(len(w.patches)))
    dm = abs(mass - o.mass()) / o.mass()
    ok = bool(np.all(err <= bar)) and masks_ok and dm <= 1e-13
    return {"case": w.name + ("_mapped" if nodes else ""), "patches": len(w.patches),
            "level0_steps": 1,
            "field_scale": scale.tolist(), "field_errors": err.tolist(), "bars": bar.tolist(),
            "masks_equal": masks_ok, "mass_rel_diff": dm, "gpu_s": t_gpu,
            "oracle_s_two_runs": t_orc, "pass": ok}


def c5link(args):
    ws = W.ensemble()
    s = int(np.argmin([w.grid.nx for w in ws]))
    w = ws[s]
    print("case", w.name, "scenario", s, args.steps, "steps", flush=True)
    t0 = time.perf_counter()
    ctx = H.Context(ws[0].params, precision=0)
    for k, x in enumerate(ws):
        ctx.add_grid(k, x.grid)
    ctx.finalize()
    for k, x in enumerate(ws):
        ctx.set_bathymetry(k, x.b)
        ctx.set_state(k, x.q)
        ctx.set_gauges(k, x.gauges)
        ctx.set_clock(k, 0.0, x.dt, 0)
    ctx.autotune()
    ctx.advance(-1.0, args.steps)
    got, mask = ctx.get_state(s), ctx.get_mask(s)
    tg, eg = ctx.read_gauges(s)
    t_gpu = time.perf_counter() - t0
    print("GPU done in %.1f s" % t_gpu, flush=True)
    runs = []

    def run(x):
        r = O.from_workload(x)
        r.advance(x.dt, args.steps)
        runs.append(r)
        print("oracle run done", flush=True)
        return [r.get_state()]

    t1 = time.perf_counter()
    exp, bars = oracle_bars(run, w, seeds=(1,))
    t_orc = time.perf_counter() - t1
    r = runs[0]
    e = field_errors(got, exp[0])
    to, eo = r.read_gauges()
    ge = float(np.abs(eg - eo).max()) / w.amplitude
    ok = bool(np.all(e <= bars[0])) and np.array_equal(mask, r.get_mask()) and ge <= TOL \
        and np.allclose(tg, to, rtol=1e-12, atol=0)
    return {"case": w.name, "scenario": s, "steps": args.steps, "field_errors": e.tolist(),
            "bars": bars[0].tolist(), "gauge_err_over_amp": ge, "masks_equal":
            bool(np.array_equal(mask, r.get_mask())), "gauge_records": int(len(tg)),
            "gpu_s": t_gpu, "oracle_s_two_runs": t_orc, "pass": ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", required=True, choices=["c5link", "c4step"])
    ap.add_argument("--steps", type=int, default=3000, help="c5link: fixed steps")
    ap.add_argument("--mapped", action="store_true", help="c4step: on the distorted mapped grid")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    out = (c5link if args.case == "c5link" else c4step)(args)
    ok = out["pass"]
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
