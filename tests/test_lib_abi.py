"""CPU checks of the boundary: the library loads and exports every symbol the header declares, and the
host-side argument checks reject bad input without touching a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mipwa.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mipwa_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mipwa_create", "mipwa_load_events", "mipwa_load_norm", "mipwa_set_params", "mipwa_eval",
                 "mipwa_eval_async", "mipwa_fit", "mipwa_integrals", "mipwa_generate"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1703_03284_amd import _lib
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_1703_03284_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_strerror_and_null_handling():
    import ctypes as C
    from paper_1703_03284_amd import _lib
    lib = _lib.load()
    assert lib.mipwa_strerror(0) == b"ok"
    assert lib.mipwa_strerror(-5) == b"non-finite likelihood"
    assert lib.mipwa_last_error(None) == b"context is NULL"
    assert lib.mipwa_eval(None, None, None) == -1
    assert lib.mipwa_create(None, 0, 0, None) == -1
    # an out-of-range precision is rejected before any device call
    out = C.c_void_p()
    assert lib.mipwa_create(None, 7, 0, C.byref(out)) == -1


def test_product_path_has_no_oracle_dependency():
    """The package must not import or reference the oracle (it is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_1703_03284_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


@pytest.mark.parametrize("name", ["kernels.hip", "host.cpp", "mipwa.cpp", "fit.cpp", "gen.cpp"])
def test_sources_present(name):
    assert os.path.exists(os.path.join(ROOT, "paper_1703_03284_amd", "csrc", name))


def test_one_hip_runtime_per_process():
    # the binding loads PyTorch's HIP runtime first, so libmipwa binds to it instead of mapping a
    # second libamdhip64 (two runtimes in one process: the second to initialise finds no GPU)
    import subprocess
    import sys
    code = ("import paper_1703_03284_amd._lib as L; L.load(); "
            "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}; "
            "print(len(maps)); print(*sorted(maps))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split()[0] == "1", r.stdout
