"""Compiles the gfx950 library libptsg.so in place (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libptsg.so")
SOURCES = ["runtime.hip", "batch.hip", "server.hip", "sweep.hip", "steps.hip", "houdayer.hip", "fused.hip"]

# Packed FP32 instructions are disabled on purpose (no float code needs them).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


PROBE = os.path.join(HERE, "rate_probe")
PROBE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    """Builds libptsg.so and the instruction-rate probe (measurement support
    for the roofline, not linked into the library)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    probe = [hipcc] + PROBE_FLAGS + ["-o", PROBE + ".tmp", os.path.join(CSRC, "rate_probe.hip")]
    if verbose:
        print(" ".join(probe), flush=True)
    subprocess.run(probe, check=True)
    os.replace(PROBE + ".tmp", PROBE)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
