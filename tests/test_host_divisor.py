"""The stream-collide kernels turn node ids into (x, y, z) with a
multiply-high and two shifts per division (common.h, invariant divisors of
Granlund and Montgomery).  The same header code, compiled for the CPU, is
checked against the hardware division for every divisor up to 65536 (edge and
random dividends up to 2^32 - 1) and two million random divisor/dividend
pairs."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="needs the ROCm clang++")
def test_invariant_division_matches_hardware(tmp_path):
    exe = str(tmp_path / "divisor_check")
    subprocess.run([CLANG, "-x", "c++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__",
                    "-D__HIP_MEMORY_SCOPE_SYSTEM=5", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "hoststub", "divisor_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
