"""Build of the HIP library libhsgn.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libhsgn.so")
SOURCES = [os.path.join(CSRC, "hsgn_api.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("hsgn_math.hpp", "hsgn_march.hpp")] + \
          [os.path.join(INCLUDE, "hsgn.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (their forms are not trusted on this target)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fused multiply-add where the compiler finds a*b+c
    "-ffp-contract=fast",
    # FP32 division and square root to ~1 ulp (the FP64 ones stay IEEE)
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile libhsgn.so for gfx950; always recompiles."""
    cmd = [HIPCC] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-o", LIB_PATH + ".tmp"] + SOURCES
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
