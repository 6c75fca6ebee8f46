"""The library's host-side model code (spline setup, evaluation and resonance tables, interval lookup,
region test) built on the CPU under AddressSanitizer and UBSan and run over models from 2 to 128 knots
with 0 to 4 resonances: every table routine writes into a heap buffer of exactly the size the library
allocates for it, so an overrun or an undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/bin/amdclang++"

pytestmark = pytest.mark.skipif(not os.path.exists(CXX), reason="needs the ROCm clang to build the host code")


def test_host_model_code_is_memory_clean(tmp_path):
    exe = str(tmp_path / "host_memory")
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1703_03284_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "host_memory.cpp"),
           os.path.join(ROOT, "paper_1703_03284_amd", "csrc", "host.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "40 models checked" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
