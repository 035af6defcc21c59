"""Benchmark of the HSGN/SWE time step on one MI355X.

A step is one accepted time step of the whole hot path (source half steps,
x and y normal solves, limiters, transverse splits, flux-difference update,
SWE switch and fix-ups, CFL control) over every cell of the workload.

Default workload: the 1024 x 1024 plane beach with an incoming SGN solitary
wave (FP64, adaptive CFL 0.9, reflecting walls, SWE transition below 0.05,
breaking latch, 16 gauges).  Inputs are synthetic (seeded generators in
paper_2606_12162_amd/workloads.py) and resident in HBM before timing starts.

Prints one JSON line: value = interior cell-updates per second over the
timed steps; roofline = the step kernel's algorithmic HBM bytes per launch
over its average launch time (HIP events on the library's stream);
cpu_baseline = the FP64 CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per FP64 cell update: read Q^n (7 x 8) and write Q^{n+1}
# (7 x 8), read the bathymetry (8), read and write the mask byte (1 + 1)
ALG_BYTES_FP64 = 7 * 8 * 2 + 8 + 2


def workload_by_name(name):
    from paper_2606_12162_amd import workloads as W
    if name == "beach":
        return [W.beach_soliton()]
    if name == "hump":
        return [W.gaussian_hump()]
    if name == "ocean":
        return [W.synthetic_ocean()]
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(ws, steps, dt):
    """The FP64 oracle as it stands, on `steps` steps of the first workload."""
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        O.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    w = ws[0]
    g = O.from_workload(w)
    t0 = time.perf_counter()
    g.advance(dt, steps)
    el = time.perf_counter() - t0
    cells = w.grid.nx * w.grid.ny
    return {"value": cells * steps / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d steps of %s (%d cell-updates), wall %.1f s"
                      % (steps, w.name, cells * steps, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="beach")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", default="",
                    help="comma-separated tile heights to time before the run; the "
                         "fastest is used for the timed steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_12162_amd import hsgn as H

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ws = workload_by_name(args.workload)
    dt = ws[0].dt
    tile_rows = args.tile_rows
    if args.sweep:
        best = None
        for th in [int(x) for x in args.sweep.split(",")]:
            c = H.from_workloads(ws, tile_rows=th)
            c.advance(dt, 5)
            c.set_timing(True)
            c.advance(dt, 50)
            ms, n = c.get_timing()
            c.close()
            us = ms / max(n, 1) * 1e3
            print("sweep: tile rows %d: step kernel %.1f us" % (th, us), file=sys.stderr, flush=True)
            if best is None or us < best[0]:
                best = (us, th)
        tile_rows = best[1]
    ctx = H.from_workloads(ws, tile_rows=tile_rows)
    cells = sum(w.grid.nx * w.grid.ny for w in ws)
    print("bench: %s, %d cells, %d work items, warmup %d, steps %d"
          % (ws[0].name, cells, ctx.work_items(), args.warmup, args.steps),
          file=sys.stderr, flush=True)

    if args.warmup:
        ctx.advance(dt, args.warmup)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(dt, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern_ms, launches = ctx.get_timing()
    ctx.set_timing(False)
    diag = ctx.diagnostics(0)

    value = cells * args.steps / el
    kavg_s = kern_ms / max(launches, 1) / 1e3
    achieved = ALG_BYTES_FP64 * cells / kavg_s / 1e9
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ws[0].name, "cells": cells, "precision": "fp64",
                   "dt": "adaptive, cfl 0.9" if dt <= 0 else "fixed %.6g" % dt,
                   "rejected_steps": diag["rejected"], "max_courant": diag["max_courant"],
                   "work_items": ctx.work_items(), "tile_rows": tile_rows or "library"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "march_kernel", "kernel_avg_us": kavg_s * 1e6,
                     "launches": launches, "alg_bytes_per_cell": ALG_BYTES_FP64},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ws, args.cpu_steps, dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
