"""The library's host-side numerical code (dense eigensolvers and QL, block-tridiagonal
solve, CholQR deflation, phi_1 by scaling and squaring, AAA poles, the aggregation
multigrid hierarchy) built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
and run on small inputs by tests/host_sanitize/check_host.cpp, which also checks each
result's defining property.  Host only: no device is touched."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_11338_amd", "csrc")
HOST_SOURCES = ["dense_host.cpp", "aaa_host.cpp", "amg_host.cpp"]


def test_host_code_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path / "check_host")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "host_sanitize", "check_host.cpp")]
    cmd += [os.path.join(CSRC, f) for f in HOST_SOURCES] + ["-o", exe, "-lpthread"]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-4000:])
    assert "0 failure(s)" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
