"""The library's host code (runtime.cpp, adjoint.cpp: handles, block tables,
graph bookkeeping, tuner, adjoint workspaces and graph caches, checkpoints)
built on the CPU against the HIP stand-in tests/hoststub/hip_stub.cpp with
AddressSanitizer, UndefinedBehaviorSanitizer and libstdc++ assertions, and
driven through the call sequences of the GPU tests and the benchmark
(tests/hoststub/drive.py).  Any heap or stack overrun, use after free,
double destroy of a stream, event or graph, or out-of-range container access
fails the test.  No GPU is used."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


def _asan_runtime():
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(not os.path.exists(CLANG), reason="needs the ROCm clang++")
def test_host_code_is_clean_under_sanitizers(tmp_path):
    rt = _asan_runtime()
    assert rt, "AddressSanitizer runtime not found"
    lib = str(tmp_path / "libhoststub.so")
    csrc = os.path.join(ROOT, "paper_2202_12147_amd", "csrc")
    cmd = [CLANG, "-x", "c++", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
           # the builtin's scope operand (system scope) outside HIP compilation
           "-D__HIP_MEMORY_SCOPE_SYSTEM=5",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-g", "-O1",
           "-fno-omit-frame-pointer", "-D_GLIBCXX_ASSERTIONS", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fPIC", "-shared",
           os.path.join(csrc, "runtime.cpp"), os.path.join(csrc, "adjoint.cpp"),
           os.path.join(ROOT, "tests", "hoststub", "hip_stub.cpp"), "-o", lib]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    work = tmp_path / "work"
    work.mkdir()
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "hoststub", "drive.py"), lib, str(work)],
                       env=env, capture_output=True, text=True, timeout=900)
    print(r.stdout[-2000:], r.stderr[-6000:])
    assert r.returncode == 0
    assert "host sequences done" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
