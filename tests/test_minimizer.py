"""The fit's BFGS minimiser (the native one behind mipwa_fit and serving) on the CPU, under
AddressSanitizer and UBSan, against objectives whose answers are known in closed form: a quadratic
(minimum, and covariance 2 H^-1 = A^-1), the same with held parameters (the conditional minimum),
Rosenbrock in 2 and 10 dimensions, the fold of a (magnitude, phase) pair with a negative magnitude
and the sign flip of its covariance, an objective that is +inf outside its domain, and the error
returns (a failing evaluation, nothing floated, a non-finite start, the iteration limit)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/bin/amdclang++"
PKG = os.path.join(ROOT, "paper_1703_03284_amd")

pytestmark = pytest.mark.skipif(not os.path.exists(CXX), reason="needs the ROCm clang to build the host code")


def test_bfgs_on_closed_form_objectives(tmp_path):
    assert os.path.exists(os.path.join(PKG, "libmipwa.so")), "build the library first (__graft_entry__.build())"
    exe = str(tmp_path / "minimizer")
    # fit.cpp is compiled in (instrumented); the rest of the library, which mipwa_fit calls, is linked
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "native", "minimizer.cpp"), os.path.join(PKG, "csrc", "fit.cpp"),
           "-L" + PKG, "-lmipwa", "-Wl,-rpath," + PKG, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "minimizer: 0 failures" in r.stdout
    shutil.rmtree(tmp_path, ignore_errors=True)
