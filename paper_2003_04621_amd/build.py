"""Compiles the gfx950 library libptsg.so in place (hipcc, no JIT cache).

Each translation unit is compiled to an object of its own, in parallel, and
the objects are linked into the shared library (every unit carries its own
device code object; no relocatable device code is needed).
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libptsg.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["runtime.hip", "batch.hip", "server.hip", "sweep.hip", "steps.hip", "houdayer.hip",
           "fused.hip", "fused_k2a.hip", "fused_k2b.hip", "fused_k3a.hip", "fused_k3b.hip",
           "gauss.hip", "gauss_fused.hip"]

# Packed FP32 instructions are disabled on purpose (no float code needs them).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _jobs() -> int:
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return min(os.cpu_count() or 1, 8)


def build(verbose: bool = False) -> str:
    """Builds libptsg.so: one hipcc per source in parallel, then one link."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src: str) -> str:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + FLAGS + inc + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    # the largest unit first, so that it does not start last
    order = sorted(SOURCES, key=lambda s: -os.path.getsize(os.path.join(CSRC, s)))
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = dict(zip(order, ex.map(compile_one, order)))
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [objs[s] for s in SOURCES]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
