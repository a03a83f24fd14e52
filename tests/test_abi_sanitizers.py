"""The library's host code built with the address and undefined-behaviour sanitizers (host
pass only; the device code is built as usual) and driven through the C ABI's argument checks
and refusal paths by tests/abi_sanitize_driver.c: the documented status for every refusal,
no sanitizer finding.  Runs without a GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    inc = os.path.join(REPO, "include")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    lib_o, drv_o, exe = (str(tmp_path / n) for n in ("rod_lib.o", "driver.o", "abi_sanitized"))
    steps = [
        # (the device code, never run here, is built without optimisation or debug information:
        # it is the slow part of the build)
        [HIPCC, "--offload-arch=gfx950", "-parallel-jobs=2", "-O1", "-Xarch_device", "-O0",
         "-Xarch_host", "-g", "-std=c++17", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", *san, "-I", inc, "-c",
         os.path.join(REPO, "paper_2509_04277_amd", "csrc", "rod_lib.hip"), "-o", lib_o],
        [HIPCC, "-x", "c", "-I", inc, "-c", os.path.join(HERE, "abi_sanitize_driver.c"), "-o", drv_o],
        [HIPCC, *san, drv_o, lib_o, "-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    # (a library the environment preloads may come before the sanitizer runtime; the HIP
    # runtime's own allocations are not this library's to answer for)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
