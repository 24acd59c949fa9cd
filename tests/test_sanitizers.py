"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host-side code, run on the CPU.

- The oracle (plain C) with the driver ``sanitize/oracle_driver.c``: every oracle entry point on
  seeded inputs of many shapes, invariants checked, leaks checked.
- The library's host code (argument validation and workspace sizing of the C ABI) with the
  driver ``sanitize/host_driver.cpp``: only the host half is instrumented (each sanitizer flag
  follows ``-Xarch_host``), and no call of the driver reaches a GPU.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    return res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(
        ["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", os.path.join(HERE, "sanitize", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "wsr_oracle.c"), "-o", exe, "-lpthread", "-lm"])
    assert "ok" in _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_validation_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_asan")
    csrc = os.path.join(ROOT, "paper_2311_03096_amd", "csrc")
    host_san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        host_san += ["-Xarch_host", flag]
    subprocess.check_call(
        [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops"] + host_san +
        [os.path.join(HERE, "sanitize", "host_driver.cpp")] +
        [os.path.join(csrc, s) for s in ("wsr_small.hip", "wsr_big.hip", "wsr_api.hip")] + ["-o", exe],
        stderr=subprocess.DEVNULL)
    # the HIP runtime's own allocations are not this code's: leak checking is off here
    assert "ok" in _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
