"""Benchmark of the HSGN/SWE time step on one MI355X.

A step is one accepted time step of the whole hot path (source half steps,
x and y normal solves, limiters, transverse splits, flux-difference update,
SWE switch and fix-ups, CFL control) over every cell of the workload.

Default workload (--workload ensemble): 48 independent source scenarios on
synthetic shelf oceans (grids of 512^2 to 1536^2 cells, 500 m to 2 km
spacing, dipole sources of 1-8 m), advanced together, one launch per step,
in the mixed FP32/FP64 form with each scenario's own fixed CFL-0.9 step.
The same ensemble is then advanced in plain FP64 over the same steps; the
line reports both rates and the gauge error of the mixed run against the
FP64 run (the FP64 kernels match the FP64 CPU oracle to 1e-11, see tests).
Other workloads: --workload hump (128^2 Gaussian hump, periodic, FP64,
adaptive), --workload beach (1024^2 plane beach, FP64, adaptive),
--workload ocean (2048^2 synthetic ocean, mixed and FP64) and --workload amr
(the ocean as a three-level patch set: 256 level-0 patches of 128^2, 1000
level-1 and 1250 level-2 patches of 16..128 cells around a circular wave;
one step is a level-0 step with its 4 + 16 substeps, a cell update is one
cell advanced one step of its own level).

Inputs are synthetic (seeded generators in paper_2606_12162_amd/workloads.py)
and resident in HBM before timing starts.  The JSON line's roofline is the
HBM one: the algorithmic bytes of a cell update (read Q^n and write Q^{n+1},
7 variables, read the bathymetry and the mask byte: 121 B in FP64, 61 B in
mixed precision) times the cells one step-kernel launch advances, over that
launch's average time (HIP events on the library's stream; in mixed
precision a "launch" is the split step: item classification, the two item
lists, and the kernels without and with the FP64 edge solve, the last on a
second stream joined back before the closing event), against 8 TB/s.  The
kernel issues far more vector ALU instructions than those bytes need, so
the vector ALU rate is reported beside it: 1259 algorithmic flops per cell
update (csrc/opcount.cpp) against 78.6 TFLOP/s (256 CUs x 64 FMA lanes x 2
flops x 2.4 GHz, unpacked FP32 and FP64) and against the 157.3 TFLOP/s of
packed FP32.  `traffic` is the HBM bytes per launch measured with rocprofv3
counters (the sum over the kernels of one launch) for the current kernel
sources (null when the sources have changed since).
After the timed steps, an untimed leg advances the workload again from its
initial state over its whole horizon (--gauge-steps, default the workload's
step count: 3000 for the ensemble) in mixed precision and in FP64 with the
same fixed steps, and reports per scenario the gauge error and the final
surface-field error of the mixed run against the FP64 run, relative to the
source amplitude.
cpu_baseline is the FP64 CPU oracle on a bounded sample of the same
workload: the median of 3 runs on the host threads given to the process, the
CPU model and core counts, and a single-thread run.

`python bench.py --copy-calibration` runs one 2 GiB device copy and nothing
else: the kernel whose FETCH_SIZE / WRITE_SIZE counters calibrate the byte
counters of the step kernel.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12      # 78.6
PACKED_FP32_PEAK_TFLOPS = 157.3
# algorithmic flops per cell update (csrc/opcount.cpp)
ALG_FLOPS = 1259
# algorithmic bytes per cell update: read Q^n and write Q^{n+1} (7 variables),
# read the bathymetry and the mask byte
ALG_BYTES = {"fp64": 7 * 8 * 2 + 8 + 1, "mixed": 7 * 4 * 2 + 4 + 1}
# what one timed step-kernel launch is
STEP_KERNELS = {"fp64": "march_kernel<fp64>",
                "mixed": "classify + lists + march_kernel<mixed> (deep items) "
                         "|| march_kernel<mixed, fp64 edges> (other items)"}
# HBM bytes per step-kernel launch from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per launch, summed over its kernels; FETCH_SIZE x 2.0 and
# WRITE_SIZE x 1.0, the factors a plain 2 GiB copy reads), per tile height,
# for the kernel sources whose digest is given; another tile height or any
# change to those sources leaves the figure null
KERNEL_SOURCES = ["hsgn_math.hpp", "hsgn_march.hpp", "hsgn_step.hpp",
                  "hsgn_step32.hip", "hsgn_step64.hip"]
MEASURED_TRAFFIC = {
    ("ensemble", "mixed"): {"digest": "dfde4759552ce4fd",
                            "tiles": {24: (1.033315e+06, 1.413443e+06), 28: (1.013762e+06, 1.414979e+06),
                                      32: (1.000020e+06, 1.417632e+06), 40: (9.815231e+05, 1.419714e+06),
                                      48: (9.704580e+05, 1.425438e+06), 56: (9.631130e+05, 1.429830e+06)}},
    ("ensemble", "fp64"): {"digest": "dfde4759552ce4fd",
                           "tiles": {40: (1.722454e+06, 2.752222e+06), 48: (1.705094e+06, 2.756582e+06),
                                     56: (1.691234e+06, 2.759149e+06), 64: (1.681060e+06, 2.761092e+06)}},
}


def kernel_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_12162_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, tile_rows, model="hsgn"):
    m = MEASURED_TRAFFIC.get((workload, precision)) if model == "hsgn" else None
    if m is None or m["digest"] != kernel_digest() or len(tile_rows) != 1:
        return None
    fw = m["tiles"].get(tile_rows[0])
    if fw is None:
        return None
    return (fw[0] * 2.0 + fw[1] * 1.0) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# mapped-grid runs (--mapped): node coordinates per scenario (patch sets:
# per patch of the scenario), or None
MAPPING = None


def make_context(H, ws, precision, tile_rows=0, gauges=True):
    ctx = H.Context(ws[0].params, tile_rows=tile_rows, precision=1 if precision == "mixed" else 0)
    for s, w in enumerate(ws):
        ctx.add_grid(s, w.grid)
    ctx.finalize()
    for s, w in enumerate(ws):
        if MAPPING is not None:
            ctx.set_mapping(s, *MAPPING[s])
        ctx.set_bathymetry(s, w.b)
        ctx.set_state(s, w.q)
        if gauges and len(w.gauges):
            ctx.set_gauges(s, w.gauges)
        if w.dt > 0:
            ctx.set_clock(s, 0.0, w.dt, 0)
    return ctx


def run(H, torch, ws, precision, steps, warmup, tile_rows=0, autotune=True):
    """Advance the workloads; returns (context, seconds, kernel ms per launch,
    launches, tile rows per level)."""
    if hasattr(ws[0], "patches"):
        return run_amr(H, torch, ws, precision, steps, warmup, tile_rows, autotune)
    ctx = make_context(H, ws, precision, tile_rows)
    rows = ctx.autotune() if autotune and not tile_rows else [tile_rows or "library"]
    dt = -1.0 if ws[0].dt > 0 else 0.0          # per-scenario fixed steps, or adaptive
    if warmup:
        ctx.advance(dt, warmup)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n = ctx.get_timing()
    ctx.set_timing(False)
    return ctx, el, ms / max(n, 1), n, rows


def run_amr(H, torch, ws, precision, steps, warmup, tile_rows=0, autotune=True):
    """Patch sets: the timed steps replay the captured level-0 step graph;
    a second, untimed-by-the-clock pass of the same number of steps with
    direct launches times every step-kernel launch with HIP events"""
    ctx, _ = H.from_amr_workloads(ws, tile_rows=tile_rows,
                                  precision=1 if precision == "mixed" else 0, nodes=MAPPING)
    rows = ctx.autotune() if autotune and not tile_rows else [tile_rows or "library"]
    if warmup:
        ctx.advance(-1.0, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(-1.0, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.set_timing(True)
    ctx.advance(-1.0, steps)
    ms, n = ctx.get_timing()
    ctx.set_timing(False)
    return ctx, el, ms / max(n, 1), n, rows


def run_adaptive(H, torch, w, steps, every, tol0, levels=2):
    """Regridded patch sets: level 0 of the ocean as given, levels 1..levels
    rebuilt every `every` level-0 steps from the surface-jump flags (the
    tolerance shrinks by 4 per level, as the jumps do with the spacing).
    Returns wall times of the whole loop and of the regrids, the cell updates
    done, the step-kernel timing and the patch counts per level."""
    ctx, _ = H.from_amr_workloads([w], precision=1)

    def regrid_all():
        for l in range(levels):
            ctx.regrid(0, l, tol=tol0 / 4.0 ** l, nbuf=2)

    regrid_all()
    ctx.advance(-1.0, 1)                      # warm-up and graph capture
    torch.cuda.synchronize()
    ctx.set_timing(True)
    updates, t_regrid, nreg = 0, 0.0, 0
    counts = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        plist = ctx.patches()
        updates += k * sum(p["nx"] * p["ny"] * 4 ** p["level"] for p in plist)
        counts.append([sum(1 for p in plist if p["level"] == l) for l in range(levels + 1)])
        ctx.advance(-1.0, k)
        done += k
        if done < steps:
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            regrid_all()
            torch.cuda.synchronize()
            t_regrid += time.perf_counter() - r0
            nreg += 1
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n = ctx.get_timing()
    ctx.set_timing(False)
    return ctx, el, t_regrid, nreg, updates, ms / max(n, 1), n, counts


def amr_updates(w):
    """cell updates of one level-0 step of a patch set"""
    return sum(p.nx * p.ny * 4 ** p.level for p in w.patches)


def host_cpu():
    """CPU model, physical cores and logical CPUs of the host, and the CPUs
    this process may run on"""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, len(cores) or None, os.cpu_count(), avail


def cpu_baseline(w, steps, nodes=None, runs=3, single_steps=None):
    """The FP64 oracle as it stands, on `steps` steps of one workload (on its
    mapped grid when node coordinates are given): the median of `runs` runs
    on the threads given to the process (OMP_NUM_THREADS, at most the CPUs
    available), and one single-thread run of `single_steps` steps."""
    import ctypes
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        O.build()
    O.lib()
    model, phys, logical, avail = host_cpu()
    threads = min(int(os.environ.get("OMP_NUM_THREADS", avail)), avail)
    gomp = ctypes.CDLL("libgomp.so.1")

    def one(n, nthreads):
        gomp.omp_set_num_threads(int(nthreads))
        g = O.from_workload(w)
        if nodes is not None:
            g.set_mapping(*nodes)
        t0 = time.perf_counter()
        g.advance(w.dt, n)
        el = time.perf_counter() - t0
        g.close()
        return w.grid.nx * w.grid.ny * n / el, el

    rates = [one(steps, threads) for _ in range(runs)]
    med = sorted(r for r, _ in rates)[runs // 2]
    single_steps = single_steps or max(1, steps // 10)
    r1, el1 = one(single_steps, 1)
    gomp.omp_set_num_threads(int(threads))
    cells = w.grid.nx * w.grid.ny
    return {"value": med, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "runs": [r for r, _ in rates], "single_thread": r1,
            "cpu_model": model, "host_physical_cores": phys, "host_logical_cpus": logical,
            "cpus_available": avail,
            "sample": "first %d steps of %s%s (%d cell-updates per run), median of %d runs, "
                      "%d threads, wall %.1f s each; single thread: %d steps in %.1f s; FP64"
                      % (steps, w.name, " (mapped)" if nodes is not None else "", cells * steps,
                         runs, threads, sorted(e for _, e in rates)[runs // 2], single_steps, el1)}


def horizon_errors(H, ws, steps):
    """Untimed: the workload from its initial state over `steps` fixed steps
    in mixed precision and in FP64; per scenario the gauge error and the
    final surface-field error (eta' over cells wet in both runs) of the mixed
    run against the FP64 run, over the source amplitude, and the relative
    error of the momenta."""
    res = {}
    for precision in ("mixed", "fp64"):
        ctx = make_context(H, ws, precision)
        ctx.advance(-1.0, steps)
        res[precision] = [(ctx.read_gauges(s)[1], ctx.get_state(s)) for s in range(len(ws))]
        ctx.close()
    gauge, field, mom = [], [], []
    for s, w in enumerate(ws):
        (ga, qa), (gb, qb) = res["mixed"][s], res["fp64"][s]
        n = min(len(ga), len(gb))
        gauge.append(float(np.abs(ga[:n] - gb[:n]).max()) / w.amplitude if n else 0.0)
        eta0 = w.params.eta0
        wet = (qa[0] > w.params.dry_tol) & (qb[0] > w.params.dry_tol)
        ea, eb = qa[0] + w.b - eta0, qb[0] + w.b - eta0
        field.append(float(np.abs(ea - eb)[wet].max()) / w.amplitude)
        m = max(float(np.abs(qb[1:3]).max()), 1e-300)
        mom.append(float(np.abs(qa[1:3] - qb[1:3]).max()) / m)
    return {"steps": steps, "records": n, "gauge_err_over_amp": gauge,
            "field_err_over_amp": field, "momentum_rel_err": mom,
            "max_gauge_err_over_amp": max(gauge), "max_field_err_over_amp": max(field)}


def gauge_error(ctx_a, ctx_b, ws):
    """max over scenarios of max |eta'_a - eta'_b| / amplitude."""
    import numpy as np
    worst = 0.0
    for s, w in enumerate(ws):
        if not len(w.gauges):
            continue
        _, ea = ctx_a.read_gauges(s)
        _, eb = ctx_b.read_gauges(s)
        n = min(len(ea), len(eb))
        worst = max(worst, float(np.abs(ea[:n] - eb[:n]).max()) / w.amplitude)
    return worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ensemble",
                    choices=["ensemble", "hump", "beach", "ocean", "amr", "amr_adaptive"])
    ap.add_argument("--regrid-every", type=int, default=10,
                    help="amr_adaptive: level-0 steps between regrids")
    ap.add_argument("--regrid-tol", type=float, default=0.004,
                    help="amr_adaptive: surface-jump tolerance on level 0 (m)")
    ap.add_argument("--regrid-levels", type=int, default=1,
                    help="amr_adaptive: refined levels rebuilt by regridding (1 or 2)")
    ap.add_argument("--precision", default="", choices=["", "mixed", "fp64"],
                    help="precision of the timed run (default: mixed, FP64 for the beach)")
    ap.add_argument("--model", default="hsgn", choices=["hsgn", "mbhsgn"],
                    help="hsgn (eq. HSGN, default) or mbhsgn (eq. mbHSGN)")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="fixed tile height (default: the library's autotuner)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's tile-height model instead of its autotuner")
    ap.add_argument("--mapped", action="store_true",
                    help="ensemble, ocean or amr on smoothly distorted mapped grids (fixed steps "
                         "0.85x; amr: nested nodes on every level)")
    ap.add_argument("--cpu-steps", type=int, default=0)
    ap.add_argument("--gauge-steps", type=int, default=-1,
                    help="steps of the untimed mixed-vs-FP64 leg (default: the workload's "
                         "horizon; 0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 2 GiB device copy (byte-counter calibration) and exit")
    ap.add_argument("--sweep", default="",
                    help="comma-separated tile heights to time before the run; the "
                         "fastest is used for the timed steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copied %d bytes" % (a.numel() * 8))
        return

    from paper_2606_12162_amd import hsgn as H
    from paper_2606_12162_amd import workloads as W
    t0 = time.perf_counter()
    if args.workload == "amr_adaptive":
        main_adaptive(args, H, W, torch)
        return
    if args.workload == "ensemble":
        ws, precision = W.ensemble(), "mixed"
    elif args.workload == "ocean":
        ws, precision = [W.synthetic_ocean()], "mixed"
    elif args.workload == "amr":
        ws, precision = [W.amr_ocean()], "mixed"
    elif args.workload == "hump":
        ws, precision = [W.gaussian_hump()], "fp64"
    else:
        ws, precision = [W.beach_soliton()], "fp64"
    amr = args.workload == "amr"
    if args.precision:
        precision = args.precision
    if args.mapped:
        global MAPPING
        if args.workload not in ("ensemble", "ocean", "amr"):
            sys.exit("--mapped applies to the ensemble, ocean and amr workloads")
        MAPPING = [W.distorted_patch_nodes(w) if amr else W.distorted_nodes(w.grid) for w in ws]
        for w in ws:
            w.dt = 0.85 * w.dt
    if args.model == "mbhsgn":
        import dataclasses
        for w in ws:
            w.params = dataclasses.replace(w.params, model=1)
            for q in ([w.q] if not amr else [p.q for p in w.patches]):
                q[4] = 0.0
                q[6] = 0.0
    cells = sum(amr_updates(w) if amr else w.grid.nx * w.grid.ny for w in ws)
    log("bench: %s x%d, %.2f M cells, precision %s, inputs generated in %.1f s"
        % (ws[0].name, len(ws), cells / 1e6, precision, time.perf_counter() - t0))

    tile_rows = args.tile_rows
    if args.sweep:
        best = None
        for th in [int(x) for x in args.sweep.split(",")]:
            c, el, kms, n, _ = run(H, torch, ws, precision, 20, 3, th)
            c.close()
            log("sweep: tile rows %d: step kernel %.1f us" % (th, kms * 1e3))
            if best is None or kms < best[0]:
                best = (kms, th)
        tile_rows = best[1]

    ctx, el, kms, launches, rows = run(H, torch, ws, precision, args.steps, args.warmup, tile_rows,
                                       not args.no_autotune)
    value = cells * args.steps / el
    # per timed step-kernel launch: the cells it advances (patch sets: the
    # launches of all levels together advance `cells` per level-0 step)
    cells_per_launch = cells * args.steps / max(launches, 1) if amr else cells
    diag = ctx.diagnostics(0)
    log("timed: %.3f ms/step, step kernel %.1f us, %.3e cell-updates/s"
        % (el * 1e3 / args.steps, kms * 1e3, value))
    tflops = ALG_FLOPS * cells_per_launch / (kms / 1e3) / 1e12
    hbm_gbs = ALG_BYTES[precision] * cells_per_launch / (kms / 1e3) / 1e9
    traffic = None if args.mapped else measured_traffic(args.workload, precision, rows, args.model)
    alg_launch = ALG_BYTES[precision] * cells_per_launch
    dtype = {"mixed": "f32+f64", "fp64": "f64"}[precision]
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
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": (ws[0].name if len(ws) == 1 else "ensemble_%d_scenarios" % len(ws))
                               + ("_mapped" if args.mapped else ""),
                   "scenarios": len(ws), "cell_updates_per_step": cells, "precision": precision,
                   "model": args.model,
                   "dt": "per-scenario fixed, cfl 0.9" if ws[0].dt > 0 else "adaptive, cfl 0.9",
                   "work_items": ctx.work_items(), "tile_rows": rows,
                   "max_courant_scenario0": diag["max_courant"]},
        "roofline": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("march_kernel_mapped<%s> (split step in mixed precision)" % precision) if args.mapped
                               else STEP_KERNELS[precision], "kernel_avg_us": kms * 1e3,
                     "launches": launches, "alg_bytes_per_cell": ALG_BYTES[precision],
                     "alg_bytes_per_launch": alg_launch,
                     "traffic_over_alg": traffic / alg_launch if traffic else None,
                     "alu": {"achieved": tflops, "unit": "TFLOP/s", "alg_flops_per_cell": ALG_FLOPS,
                             "peak_fma": ALU_PEAK_TFLOPS, "frac_fma": tflops / ALU_PEAK_TFLOPS,
                             "peak_packed_fp32": PACKED_FP32_PEAK_TFLOPS,
                             "frac_packed_fp32": tflops / PACKED_FP32_PEAK_TFLOPS}},
    }
    if precision == "mixed" and not args.no_fp64:
        ctx64, el64, kms64, _, rows64 = run(H, torch, ws, "fp64", args.steps, args.warmup,
                                            tile_rows, not args.no_autotune)
        hbm64 = ALG_BYTES["fp64"] * cells_per_launch / (kms64 / 1e3) / 1e9
        traffic64 = None if args.mapped else measured_traffic(args.workload, "fp64", rows64, args.model)
        alg64 = ALG_BYTES["fp64"] * cells_per_launch
        out["fp64_plain"] = {"value": cells * args.steps / el64,
                             "ms_per_step": el64 * 1e3 / args.steps,
                             "kernel_avg_us": kms64 * 1e3, "tile_rows": rows64,
                             "roofline": {"bound": "hbm", "achieved": hbm64, "peak": HBM_PEAK_GBS,
                                          "unit": "GB/s", "frac": hbm64 / HBM_PEAK_GBS,
                                          "alg_bytes_per_cell": ALG_BYTES["fp64"],
                                          "traffic": traffic64,
                                          "traffic_over_alg": traffic64 / alg64 if traffic64 else None,
                                          "alu_tflops": ALG_FLOPS * cells_per_launch / (kms64 / 1e3) / 1e12}}
        out["mixed_over_fp64"] = value / out["fp64_plain"]["value"]
        out["gauge_err_over_amp_timed_run"] = gauge_error(ctx, ctx64, ws)
        log("fp64: %.3f ms/step; mixed/fp64 %.2fx; gauge error / amplitude over the timed run %.2e"
            % (out["fp64_plain"]["ms_per_step"], out["mixed_over_fp64"],
               out["gauge_err_over_amp_timed_run"]))
        ctx64.close()
    ctx.close()
    gsteps = args.gauge_steps if args.gauge_steps >= 0 else ws[0].steps
    if precision == "mixed" and not args.no_fp64 and gsteps > 0 and not amr and ws[0].dt > 0:
        t1 = time.perf_counter()
        he = horizon_errors(H, ws, gsteps)
        out["horizon"] = he
        out["gauge_err_over_amp"] = he["max_gauge_err_over_amp"]
        log("horizon leg: %d steps, %.1f s; gauge error / amplitude max %.2e, field error / "
            "amplitude max %.2e" % (gsteps, time.perf_counter() - t1, he["max_gauge_err_over_amp"],
                                    he["max_field_err_over_amp"]))
    if not args.no_cpu_baseline:
        steps = args.cpu_steps or (40 if args.workload == "ensemble" else 20)
        # patch sets: the oracle on the level-0 ocean grid of the same set
        base = W.synthetic_ocean() if amr else ws[0]
        nodes = None
        if MAPPING is not None:
            nodes = W.distorted_nodes(base.grid) if amr else MAPPING[0]
        out["cpu_baseline"] = cpu_baseline(base, steps, nodes)
    print(json.dumps(out), flush=True)


def main_adaptive(args, H, W, torch):
    import dataclasses
    full = W.amr_ocean()
    w = dataclasses.replace(full, patches=[p for p in full.patches if p.level == 0])
    log("bench: %s, level 0 only (%d patches), %d level(s) regridded every %d steps, "
        "tolerance %.4g m" % (full.name, len(w.patches), args.regrid_levels, args.regrid_every,
                              args.regrid_tol))
    ctx, el, t_reg, nreg, updates, kms, launches, counts = run_adaptive(
        H, torch, w, args.steps, args.regrid_every, args.regrid_tol, args.regrid_levels)
    value = updates / el
    cells_per_launch = updates / max(launches, 1)
    tflops = ALG_FLOPS * cells_per_launch / (kms / 1e3) / 1e12
    hbm_gbs = ALG_BYTES["mixed"] * cells_per_launch / (kms / 1e3) / 1e9
    log("timed: %.3f ms/step incl. regrids, %d regrids of %.1f ms, %.3e cell-updates/s; "
        "patches per level %s .. %s" % (el * 1e3 / args.steps, nreg,
                                        t_reg * 1e3 / max(nreg, 1), value, counts[0], counts[-1]))
    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": full.name + "_regridded", "precision": "mixed",
                   "regrid_every": args.regrid_every, "regrid_tol_level0": args.regrid_tol,
                   "regrid_levels": args.regrid_levels,
                   "patches_per_level_first": counts[0], "patches_per_level_last": counts[-1]},
        "regrid": {"count": nreg, "ms_mean": t_reg * 1e3 / max(nreg, 1),
                   "share_of_wall": t_reg / el,
                   "stepping_only_value": updates / max(el - t_reg, 1e-12)},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": ALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / ALU_PEAK_TFLOPS, "traffic": None,
                     "kernel": STEP_KERNELS["mixed"], "kernel_avg_us": kms * 1e3,
                     "launches": launches,
                     "hbm": {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": hbm_gbs / HBM_PEAK_GBS}},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
