"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU, of
the oracle and of the host-side entry points that need no device (the cost
of a packing, the host lower bound, the checks of model loading).  Each is
driven over seeded random and edge inputs by a small program and must run
clean.  Needs gcc/g++ with the sanitizer runtimes; no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", *SAN, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "vsbpp_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert "0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not available")
def test_host_calls_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
          os.path.join(ROOT, "paper_1602_08735_amd", "csrc", "host_calls.cpp"),
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    # leak checking is off here: the HIP runtime's own start-up allocations
    # are not this code's
    r = _run([exe, str(tmp_path)], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    assert "0 failures" in r.stdout
