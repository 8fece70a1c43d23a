"""AddressSanitizer / UndefinedBehaviorSanitizer runs of the host code (no GPU
needed): the CPU oracle driven through every exported routine
(sanitize_oracle.c), and the host side of libptsg's C ABI -- argument
checks, host-only planners, the round-trip summary, the host acceptance
decision and the creation failure paths without a device
(sanitize_runtime.cpp).  Leak detection is on; UBSan does not recover, so
any report fails the test."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    p = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    report = p.stdout + p.stderr
    assert p.returncode == 0, report[-4000:]
    assert "Sanitizer" not in report and "runtime error" not in report, report[-4000:]
    return report


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    srcs = [os.path.join(HERE, "sanitize_oracle.c")] + [
        os.path.join(ROOT, "oracle", f) for f in ("ea_oracle.c", "gauss_oracle.c", "enum.c")]
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe] + srcs + ["-lquadmath", "-lm"], check=True)
    assert "sanitized oracle run complete" in _run(exe)


def test_runtime_host_side_under_address_and_ub_sanitizers(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_2003_04621_amd import build as B
    inc = ["-I", os.path.join(ROOT, "include"), "-I", B.CSRC]
    # sanitizers on the host side only: device code is compiled as usual
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"] + san + inc

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.run([hipcc] + flags + ["-c", "-o", obj, os.path.join(B.CSRC, src)],
                       check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    drv = str(tmp_path / "driver.o")
    subprocess.run([hipcc, "--offload-host-only", "-O1", "-g", "-std=c++17"] + san + inc +
                   ["-x", "hip", "-c", "-o", drv, os.path.join(HERE, "sanitize_runtime.cpp")],
                   check=True, capture_output=True)
    exe = str(tmp_path / "sanitize_runtime")
    subprocess.run([hipcc, "--offload-arch=gfx950"] + san[:4] + objs + [drv, "-o", exe],
                   check=True, capture_output=True)
    assert "sanitized runtime host checks complete" in _run(exe)
