"""ctypes declarations of libmipwa (include/mipwa.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MIPWA_LIB") or os.path.join(_HERE, "libmipwa.so")

MIPWA_FP64, MIPWA_MIXED = 0, 1
STATUS = {0: "MIPWA_OK", -1: "MIPWA_E_INVAL", -2: "MIPWA_E_NOMEM", -3: "MIPWA_E_HIP", -4: "MIPWA_E_STATE",
          -5: "MIPWA_E_DOMAIN", -6: "MIPWA_E_NOCONV", -7: "MIPWA_E_CANCELLED", -8: "MIPWA_E_BUSY"}


class ResC(C.Structure):
    _fields_ = [("spin", C.c_int), ("mass", C.c_double), ("width", C.c_double), ("radius", C.c_double)]


class ModelC(C.Structure):
    _fields_ = [("M", C.c_double), ("m1", C.c_double), ("m2", C.c_double), ("m3", C.c_double),
                ("rD", C.c_double), ("n_knots", C.c_int), ("knots", C.POINTER(C.c_double)),
                ("n_res", C.c_int), ("res", C.POINTER(ResC))]


class FitOptsC(C.Structure):
    _fields_ = [("tol_edm", C.c_double), ("max_iter", C.c_int), ("hessian", C.c_int)]


class FitInfoC(C.Structure):
    _fields_ = [("nll", C.c_double), ("edm", C.c_double), ("n_iter", C.c_int), ("n_eval", C.c_int),
                ("status", C.c_int)]


class ServeStatsC(C.Structure):
    _fields_ = [("fits_per_s", C.c_double), ("p50_s", C.c_double), ("p99_s", C.c_double),
                ("n_done", C.c_longlong), ("n_active", C.c_longlong), ("n_queued", C.c_longlong),
                ("peak_bytes", C.c_longlong), ("steps", C.c_longlong), ("mean_batch", C.c_double),
                ("step_device_s", C.c_double), ("device_busy", C.c_double)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64 = C.c_longlong

SIGNATURES = {
    "mipwa_create": (C.c_int, [C.POINTER(ModelC), C.c_int, C.c_int, C.POINTER(_P)]),
    "mipwa_destroy": (None, [_P]),
    "mipwa_last_error": (C.c_char_p, [_P]),
    "mipwa_strerror": (C.c_char_p, [C.c_int]),
    "mipwa_n_params": (C.c_int, [_P]),
    "mipwa_set_swave_form": (C.c_int, [_P, C.c_int]),
    "mipwa_set_norm_mode": (C.c_int, [_P, C.c_int]),
    "mipwa_load_events": (C.c_int, [_P, _D, _D, _D, _I64]),
    "mipwa_load_norm": (C.c_int, [_P, _D, _D, _D, _D, _I64]),
    "mipwa_set_eff_table": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int, C.c_int, C.c_double, C.c_double]),
    "mipwa_set_fixed": (C.c_int, [_P, C.POINTER(C.c_ubyte), C.c_int]),
    "mipwa_set_params": (C.c_int, [_P, _D, C.c_int]),
    "mipwa_eval": (C.c_int, [_P, _D, _D]),
    "mipwa_eval_async": (C.c_int, [_P, _P, _P]),
    "mipwa_eval_noalloc": (C.c_int, [_P, _P, _P]),
    "mipwa_integrals": (C.c_int, [_P, C.c_int, _D]),
    "mipwa_fit_fractions": (C.c_int, [_P, _D]),
    "mipwa_fit": (C.c_int, [_P, C.POINTER(FitOptsC), _D, _D, C.POINTER(FitInfoC)]),
    "mipwa_generate": (C.c_int, [_P, _D, C.c_int, C.c_ulonglong, C.c_double, _I64, _D, _D,
                                 C.POINTER(C.c_int), C.POINTER(_I64)]),
    "mipwa_density_max": (C.c_int, [_P, _D, C.c_int, C.c_ulonglong, _I64, _D]),
    "mipwa_toy": (C.c_int, [_P, _D, C.c_int, C.c_ulonglong, _I64, _I64, _D, _D, _D]),
    "mipwa_last_timing": (C.c_int, [_P, _D, _D]),
    "mipwa_set_launch": (C.c_int, [_P, C.c_int, C.c_int]),
    "mipwa_set_timing": (C.c_int, [_P, C.c_int]),
    "mipwa_read_bandwidth": (C.c_int, [C.c_int, _I64, C.c_int, _D]),
    "mipwa_timing_stats": (C.c_int, [_P, C.POINTER(_I64), _D, _D]),
    "mipwa_server_create": (C.c_int, [C.c_int, C.c_int, C.c_size_t, C.POINTER(_P)]),
    "mipwa_server_set_norm": (C.c_int, [_P, _D, _D, _D, _I64]),
    "mipwa_server_submit": (C.c_int, [_P, C.POINTER(ModelC), _D, _D, _I64, _D, C.POINTER(C.c_ubyte),
                                      C.POINTER(FitOptsC), C.POINTER(_I64)]),
    "mipwa_server_submit_borrowed": (C.c_int, [_P, C.POINTER(ModelC), _D, _D, _I64, _D, C.POINTER(C.c_ubyte),
                                               C.POINTER(FitOptsC), C.POINTER(_I64)]),
    "mipwa_server_poll": (C.c_int, [_P, _I64, _D, C.POINTER(FitInfoC), _D]),
    "mipwa_server_wait": (C.c_int, [_P, _I64, C.c_double, _D, C.POINTER(FitInfoC), _D]),
    "mipwa_server_cancel": (C.c_int, [_P, _I64]),
    "mipwa_server_stats": (C.c_int, [_P, C.POINTER(ServeStatsC)]),
    "mipwa_server_last_error": (C.c_char_p, [_P]),
    "mipwa_server_destroy": (None, [_P]),
}

_lib = None


def _bind_torch_runtime():
    """Load PyTorch's HIP runtime before libmipwa when PyTorch is installed.

    PyTorch carries its own libamdhip64 with the same soname as ROCm's.  Loaded first, it satisfies
    libmipwa's dependency, so the process holds one HIP runtime and device pointers and streams pass
    between PyTorch and libmipwa.  Loaded the other way round, the process would hold two runtimes
    and the second to initialise would find no GPU.
    """
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load():
    """Load libmipwa.so from the package directory; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_1703_03284_amd.build)")
    _bind_torch_runtime()
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None
