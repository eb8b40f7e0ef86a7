"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The library is compiled with both sanitizers on its host code only (device code as usual), and
tests/host_sanitizer_driver.cpp, built with the same sanitizers, calls every entry point that runs
without a GPU: parameter validation and workspace sizing over a sweep of shapes, plan creation with
invalid arguments, NULL plans, error strings.  Any sanitizer report or failed check fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.timeout(600)
def test_host_entry_points_under_asan_and_ubsan(tmp_path):
    if not (shutil.which(HIPCC) or os.path.exists(HIPCC)) or not os.path.exists(CLANG):
        pytest.skip("ROCm compilers not found")
    lib = tmp_path / "librecon_san.so"
    src = os.path.join(ROOT, "paper_1504_02591_amd", "csrc", "recon_api.hip")
    inc = os.path.join(ROOT, "include")
    # sanitizers on the host pass only: each -fsanitize= follows -Xarch_host
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    f"-I{inc}", "-o", str(lib), src, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
                    "-lrocprofiler-sdk-roctx"], check=True, capture_output=True, timeout=540)
    drv = tmp_path / "driver"
    subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    f"-I{inc}", "-o", str(drv), os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp"),
                    f"-L{tmp_path}", "-lrecon_san", f"-Wl,-rpath,{tmp_path}", "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True, capture_output=True, timeout=120)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"     # the HIP runtime keeps its allocations
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([str(drv)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
