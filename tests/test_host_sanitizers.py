"""The host-only FP64 code (the mass-spring solver and the wing-load
transpose, include/fsi_ms.h) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no device code) and driven through every
entry point, the error paths included, by tests/native/host_driver.cpp: no
invalid access, no undefined behaviour, no leak, every call as documented."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_08642_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-static-libasan", "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "structure.cpp"), os.path.join(CSRC, "loads.cpp"),
           os.path.join(ROOT, "tests", "native", "host_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr
