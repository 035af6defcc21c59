"""Build of the HIP library libhsgn.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libhsgn.so")
SOURCES = [os.path.join(CSRC, f) for f in ("hsgn_step64.hip", "hsgn_step32.hip",
                                            "hsgn_step64amr.hip", "hsgn_step32amr.hip",
                                            "hsgn_amr.hip", "hsgn_api.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("hsgn_math.hpp", "hsgn_march.hpp", "hsgn_step.hpp",
                                           "hsgn_amr.hpp")] + [os.path.join(INCLUDE, "hsgn.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions (their forms are not trusted on this target)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 division and square root to ~1 ulp (the FP64 ones stay IEEE)
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-Wno-unused-result",
]
# per-source floating-point contraction: the patch-set kernels (ghost
# interpolation, refluxing, averaging) round every product and sum
# separately; the step kernels of both precisions and the host code may fuse
# products into sums
CONTRACT = {"hsgn_amr.hip": "-ffp-contract=off"}
BUILD_DIR = os.path.join(HERE, "_build")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile libhsgn.so for gfx950; always recompiles (sources in parallel)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, procs = [], []
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 8)
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        contract = CONTRACT.get(os.path.basename(src), "-ffp-contract=fast")
        cmd = [HIPCC] + FLAGS + [contract, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        while len([p for p in procs if p.poll() is None]) >= jobs:
            procs[[p.poll() is None for p in procs].index(True)].wait()
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, p.args)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB_PATH + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def stale() -> bool:
    if not os.path.exists(LIB_PATH):
        return True
    t = os.path.getmtime(LIB_PATH)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
