"""Builds the HIP library libradsort.so for gfx950 in-tree (hipcc, no JIT)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libradsort.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# The ordering-check build (RS_DEBUG_ORDER): the same library with the check of
# RADSORT_F_DEBUG_ORDER compiled in; the product library has none of it.
DEBUG_ORDER_LIB = os.path.join(HERE, "_lib_debug_order", "libradsort.so")


def _command(out: str, defines=()) -> list:
    return [HIPCC, *FLAGS, *(f"-D{d}" for d in defines), "-o", out,
            os.path.join(CSRC, "radsort.hip")]


def build(verbose: bool = False, debug_order: bool = True) -> str:
    """Compile csrc/radsort.hip into _lib/libradsort.so (always recompiles), and
    the ordering-check build beside it (both compilations run at once)."""
    jobs = [(LIB_PATH, ())]
    if debug_order:
        jobs.append((DEBUG_ORDER_LIB, ("RS_DEBUG_ORDER",)))
    procs = []
    for out, defines in jobs:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        cmd = _command(out + ".tmp", defines)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((out, cmd, subprocess.Popen(cmd)))
    failed = [cmd for _, cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    for out, _, _ in procs:
        os.replace(out + ".tmp", out)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True, debug_order="--no-debug-order" not in sys.argv)
    print(LIB_PATH)
    sys.exit(0)
