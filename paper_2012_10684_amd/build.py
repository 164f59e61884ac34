"""Build libts.so (the HIP library behind include/ts.h) for gfx950 in-tree.

Every kernel source and the C ABI are compiled by hipcc into objects (one
hipcc process per source, in parallel) and linked into one shared library
next to this file.  Packed-FP32 instructions are disabled (-packed-fp32-ops) and
floating-point contraction is off, so each FP32 expression is evaluated
exactly as written (the search re-evaluates FP32 keys and relies on
getting the same bits).
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libts.so")
ARCH = os.environ.get("TS_OFFLOAD_ARCH", "gfx950")

COMPILE = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]
LINK = ["-shared", "-fPIC", f"--offload-arch={ARCH}"]
OBJDIR = os.path.join(HERE, "_build")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _filter(stderr: str) -> str:
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src).replace(".hip", ".o"))
    cmd = [hipcc()] + COMPILE + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = _filter(p.stderr)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({p.returncode}):\n{err}")
    if verbose and err:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source (always recompiles) and link libts.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    n = jobs or max(1, min(len(srcs), 8, len(os.sched_getaffinity(0))))
    with concurrent.futures.ThreadPoolExecutor(n) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + LINK + ["-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc link failed ({p.returncode}):\n{_filter(p.stderr)}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
