"""The library's host-side planning code under AddressSanitizer and UndefinedBehaviorSanitizer.

The row plan (colouring, XCD parts, row order, workgroup partition, long-row
chunks) and the augmented assembly run on the host at create.  Here every
library source is compiled for the host only (no device code), with both
sanitizers instrumenting the host code, and linked into a driver that calls
gabp_plan_rows and gabp_plan_augmented on valid and malformed inputs
(tests/host_sanitize/driver.cpp).  Any out-of-bounds access, use after free,
signed overflow, misaligned access or the like ends the driver with a
sanitizer report; the test requires a clean exit.  No GPU is used.
"""
import concurrent.futures
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0811_2518_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


def _sources():
    from paper_0811_2518_amd import build
    return build.SOURCES


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_planning_code_is_clean_under_sanitizers(tmp_path):
    common = ["--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
              *SANITIZE, "-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([HIPCC, *common, "-c", os.path.join(CSRC, src), "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, _sources()))
    drv_obj = str(tmp_path / "driver.o")
    r = subprocess.run([HIPCC, *common, "-x", "hip", "-c", os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"),
                        "-o", drv_obj], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "driver")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *SANITIZE, "-o", exe, drv_obj, *objs], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "ok: 0 failure(s)" in out
