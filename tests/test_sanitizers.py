"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle (every whole-matrix entry point, on designed corner-case blocks and
every tunable rate) and the library's host-side argument checks (shapes and
leading dimensions at and beyond their limits).  Built with gcc/g++ into a
temporary directory and run as child processes; any out-of-bounds access,
leak or undefined operation makes the run fail."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build_and_run(cmd, exe):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, f"build failed:\n{res.stderr[-2000:]}"
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})
    assert run.returncode == 0, f"sanitizer run failed:\n{run.stdout[-1000:]}\n{run.stderr[-3000:]}"
    return run.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    out = build_and_run(["gcc", *SAN, "-ffp-contract=off", "-fopenmp", "-o", exe,
                         os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"),
                         os.path.join(ROOT, "oracle", "blaz_oracle.c"), "-lm"], exe)
    assert "ok" in out


def test_host_validation_under_sanitizers(tmp_path):
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("HIP headers not installed")
    exe = str(tmp_path / "validate_san")
    out = build_and_run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                         "-I", os.path.join(ROOT, "include"),
                         "-I", os.path.join(ROOT, "paper_2202_13007_amd", "csrc"), "-o", exe,
                         os.path.join(ROOT, "tests", "sanitize", "validate_main.cpp")], exe)
    assert "ok" in out
