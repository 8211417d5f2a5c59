"""libsfrde's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is compiled with the sanitizers on its host part (argument
validation, plan-independent helpers, the C ABI entry points; device code is
built as usual and never launched) and linked with a C driver that exercises
every validation path and the host helpers over their range
(tests/sanitize/host_driver.c). Any sanitizer report, or a wrong return code,
fails the test. Runs on the CPU only (about a minute, most of it the device
code's compile)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2003_13569_amd", "csrc", "sfrde.hip")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_driver.c")

pytestmark = pytest.mark.slow


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not found")


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    hipcc = _hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    lib_obj = str(tmp_path / "sfrde_host.o")
    drv_obj = str(tmp_path / "driver.o")
    exe = str(tmp_path / "driver")
    inc = ["-I", os.path.join(ROOT, "include")]
    dev = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument"]
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", *dev, *san, *inc, "-c", SRC, "-o", lib_obj],
                   check=True, capture_output=True, text=True)
    subprocess.run([hipcc, "-O1", "-g", "-x", "c", *san, *inc, "-c", DRIVER, "-o", drv_obj],
                   check=True, capture_output=True, text=True)
    subprocess.run([hipcc, *san, drv_obj, lib_obj, "-o", exe], check=True, capture_output=True,
                   text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    assert "host driver: 0 failures" in out, out
