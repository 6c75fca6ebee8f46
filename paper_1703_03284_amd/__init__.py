"""MI355X engine for the unbinned MIPWA likelihood of D+ -> h- h+ h+ (see include/mipwa.h).

Thin Python binding of libmipwa: every step of the likelihood, its gradient, the fit and toy
generation runs in the library (HIP kernels on gfx950 plus its FP64 host finish); this module only
marshals arguments.  PyTorch is used only for device memory and streams (torch_nll.py).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L

__all__ = ["Context", "Server", "MipwaError", "Resonance", "FitResult", "FP64", "MIXED", "context_for"]

FP64, MIXED = L.MIPWA_FP64, L.MIPWA_MIXED
SWAVE_POLAR, SWAVE_CARTESIAN, SWAVE_ISOBAR = 0, 1, 2
NORM_POINTS, NORM_QFORM = 0, 1


class MipwaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{L.STATUS.get(status, status)}: {message}")
        self.status = status


@dataclass(frozen=True)
class Resonance:
    spin: int
    mass: float
    width: float
    radius: float


@dataclass
class FitResult:
    theta: np.ndarray
    cov: np.ndarray
    nll: float
    edm: float
    n_iter: int
    n_eval: int
    status: int

    @property
    def sigma(self) -> np.ndarray:
        return np.sqrt(np.maximum(np.diag(self.cov), 0.0))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _ModelHolder:
    """Keeps the C model struct and the arrays it points to alive."""

    def __init__(self, M, m1, m2, m3, rD, knots, resonances):
        self.knots = _f64(knots)
        self.res = (L.ResC * max(len(resonances), 1))()
        for i, r in enumerate(resonances):
            self.res[i] = L.ResC(int(r.spin), float(r.mass), float(r.width), float(r.radius))
        self.c = L.ModelC(float(M), float(m1), float(m2), float(m3), float(rD), len(self.knots),
                          self.knots.ctypes.data_as(L._D), len(resonances),
                          C.cast(self.res, C.POINTER(L.ResC)))


class Context:
    """One likelihood (events + normalisation points + model) on one GPU."""

    def __init__(self, M, m1, m2, m3, rD, knots, resonances, precision=FP64, device=0):
        self._lib = L.load()
        self._model = _ModelHolder(M, m1, m2, m3, rD, knots, resonances)
        h = C.c_void_p()
        rc = self._lib.mipwa_create(C.byref(self._model.c), int(precision), int(device), C.byref(h))
        if rc != 0:
            raise MipwaError(rc, "mipwa_create: " + self._lib.mipwa_strerror(rc).decode())
        self._h = h
        self.n_knots = len(self._model.knots)
        self.n_res = len(resonances)
        self.n_params = self._lib.mipwa_n_params(h)
        self.precision = precision
        self._eval_buffers()

    def _eval_buffers(self):
        # theta and gradient buffers with their ctypes pointers made once: building a pointer from an
        # array costs several microseconds, a noticeable share of one evaluation
        n = self.n_params
        self._th_buf, self._g_buf = np.empty(n), np.empty(n)
        self._th_ptr, self._g_ptr = L.dptr(self._th_buf), L.dptr(self._g_buf)
        self._nll = C.c_double()
        self._nll_ref = C.byref(self._nll)

    # -- plumbing
    def _check(self, rc, what):
        if rc != 0:
            raise MipwaError(rc, f"{what}: {self._lib.mipwa_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mipwa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- data
    def load_events(self, s12, s13, eff=None):
        s12, s13 = _f64(s12), _f64(s13)
        e = None if eff is None else _f64(eff)
        self._check(self._lib.mipwa_load_events(self._h, L.dptr(s12), L.dptr(s13), L.dptr(e), len(s12)),
                    "load_events")

    def load_norm(self, s12, s13, w, eff=None):
        s12, s13, w = _f64(s12), _f64(s13), _f64(np.broadcast_to(w, np.shape(s12)))
        e = None if eff is None else _f64(eff)
        self._check(self._lib.mipwa_load_norm(self._h, L.dptr(s12), L.dptr(s13), L.dptr(w), L.dptr(e), len(s12)),
                    "load_norm")

    def set_eff_table(self, table, lo, hi):
        t = np.ascontiguousarray(table, dtype=np.float32)
        nx, ny = t.shape
        self._check(self._lib.mipwa_set_eff_table(self._h, t.ctypes.data_as(C.POINTER(C.c_float)), nx, ny,
                                                  float(lo), float(hi)), "set_eff_table")

    def set_norm_mode(self, mode):
        """NORM_POINTS (default) or NORM_QFORM (per-cell moments while the shapes are fixed)."""
        self._check(self._lib.mipwa_set_norm_mode(self._h, int(mode)), "set_norm_mode")

    def set_swave_form(self, form):
        """SWAVE_POLAR (default), SWAVE_CARTESIAN or SWAVE_ISOBAR (two-knot model); resets theta and
        the fixed mask, and changes n_params."""
        self._check(self._lib.mipwa_set_swave_form(self._h, int(form)), "set_swave_form")
        self.n_params = self._lib.mipwa_n_params(self._h)
        self._eval_buffers()

    def set_fixed(self, fixed):
        f = np.ascontiguousarray(fixed, dtype=np.uint8)
        self._check(self._lib.mipwa_set_fixed(self._h, f.ctypes.data_as(C.POINTER(C.c_ubyte)), len(f)), "set_fixed")

    def set_params(self, theta):
        t = _f64(theta)
        self._check(self._lib.mipwa_set_params(self._h, L.dptr(t), len(t)), "set_params")

    def set_launch(self, blocks=0, waves=0):
        self._check(self._lib.mipwa_set_launch(self._h, int(blocks), int(waves)), "set_launch")

    # -- evaluation
    def eval(self, theta=None, raise_domain=True):
        """(-2 ln L, gradient) at theta (or the current parameters)."""
        if theta is not None:
            if np.shape(theta) != self._th_buf.shape:
                self.set_params(theta)  # reports the length mismatch
            self._th_buf[:] = theta
            self._check(self._lib.mipwa_set_params(self._h, self._th_ptr, self.n_params), "set_params")
        rc = self._lib.mipwa_eval(self._h, self._nll_ref, self._g_ptr)
        g = self._g_buf.copy()
        if rc == -5 and not raise_domain:
            return float("inf"), g
        self._check(rc, "eval")
        return self._nll.value, g

    def eval_async(self, stream_handle: int, d_out_ptr: int):
        """Enqueue an evaluation on a HIP stream; [nll, grad...] lands at the device pointer d_out_ptr."""
        self._check(self._lib.mipwa_eval_async(self._h, C.c_void_p(stream_handle), C.c_void_p(d_out_ptr)),
                    "eval_async")

    def eval_noalloc(self, stream_handle: int, d_out_ptr: int):
        """As eval_async, with the evaluation's scratch in the library's static per-GPU array: no device
        memory is allocated (point-sweep normalisation only; calls that overlap on one GPU race)."""
        self._check(self._lib.mipwa_eval_noalloc(self._h, C.c_void_p(stream_handle), C.c_void_p(d_out_ptr)),
                    "eval_noalloc")

    def timing(self):
        """(device ms of the whole evaluation, device ms of the streaming kernel) of the last timed
        evaluations (NaN for a figure they did not record; see set_timing)."""
        a, b = C.c_double(), C.c_double()
        self._check(self._lib.mipwa_last_timing(self._h, C.byref(a), C.byref(b)), "last_timing")
        return a.value, b.value

    def set_timing(self, period=1):
        """Device timing from HIP events on the evaluation stream of every period-th evaluation (0: off);
        timed evaluations alternately record the whole evaluation and the streaming kernel."""
        self._check(self._lib.mipwa_set_timing(self._h, int(period)), "set_timing")

    def timing_stats(self):
        """(timed evaluations, mean device ms of the whole evaluation, mean ms of the streaming kernel)."""
        n, a, b = C.c_longlong(), C.c_double(), C.c_double()
        self._check(self._lib.mipwa_timing_stats(self._h, C.byref(n), C.byref(a), C.byref(b)), "timing_stats")
        return n.value, a.value, b.value

    def integrals(self, with_eff=True, theta=None):
        if theta is not None:
            self.set_params(theta)
        K = self.n_res + 1
        out = np.empty(2 * K * K)
        self._check(self._lib.mipwa_integrals(self._h, int(bool(with_eff)), L.dptr(out)), "integrals")
        return (out[0::2] + 1j * out[1::2]).reshape(K, K)

    def fit_fractions(self, theta=None):
        if theta is not None:
            self.set_params(theta)
        K = self.n_res + 1
        out = np.empty(K * K)
        self._check(self._lib.mipwa_fit_fractions(self._h, L.dptr(out)), "fit_fractions")
        return out.reshape(K, K)

    def fit(self, theta0, fixed=None, tol_edm=1e-6, max_iter=1000, hessian=True, raise_noconv=True):
        if fixed is not None:
            self.set_fixed(fixed)
        th = _f64(theta0).copy()
        cov = np.zeros((self.n_params, self.n_params))
        info = L.FitInfoC()
        opts = L.FitOptsC(float(tol_edm), int(max_iter), int(bool(hessian)))
        rc = self._lib.mipwa_fit(self._h, C.byref(opts), L.dptr(th), L.dptr(cov), C.byref(info))
        if not (rc == -6 and not raise_noconv):
            self._check(rc, "fit")
        return FitResult(th, cov, info.nll, info.edm, info.n_iter, info.n_eval, info.status)

    # -- toy generation
    def generate(self, theta, n, seed, fmax):
        t = _f64(theta)
        s12, s13 = np.empty(n), np.empty(n)
        exc, ncand = C.c_int(), C.c_longlong()
        self._check(self._lib.mipwa_generate(self._h, L.dptr(t), len(t), int(seed), float(fmax), int(n),
                                             L.dptr(s12), L.dptr(s13), C.byref(exc), C.byref(ncand)), "generate")
        return s12, s13, bool(exc.value), int(ncand.value)

    def density_max(self, theta, seed, n_probe):
        t = _f64(theta)
        out = C.c_double()
        self._check(self._lib.mipwa_density_max(self._h, L.dptr(t), len(t), int(seed), int(n_probe),
                                                C.byref(out)), "density_max")
        return out.value

    def toy(self, theta, n, seed, n_probe=1_000_000):
        """Accept-reject toy sample of n points (mipwa_toy): fmax = 1.5 x the largest density over
        n_probe inside-candidates of key seed + 1000, doubled and redrawn while exceeded."""
        t = _f64(theta)
        s12, s13 = np.empty(n), np.empty(n)
        fmax = C.c_double()
        self._check(self._lib.mipwa_toy(self._h, L.dptr(t), len(t), int(seed), int(n_probe), int(n),
                                        L.dptr(s12), L.dptr(s13), C.byref(fmax)), "toy")
        return s12, s13, fmax.value


def read_bandwidth(device=0, nbytes=1 << 30, reps=10) -> float:
    """Measured streaming-read ceiling of the GPU in GB/s (mipwa_read_bandwidth)."""
    lib = L.load()
    out = C.c_double()
    rc = lib.mipwa_read_bandwidth(int(device), int(nbytes), int(reps), C.byref(out))
    if rc != 0:
        raise MipwaError(rc, "mipwa_read_bandwidth")
    return out.value


def context_for(decay, knots, resonances, precision=FP64, device=0) -> Context:
    """Context from any object with M, m1, m2, m3, rD attributes and resonance objects with spin, mass,
    width, radius attributes."""
    return Context(decay.M, decay.m1, decay.m2, decay.m3, decay.rD, knots,
                   [Resonance(r.spin, r.mass, r.width, r.radius) for r in resonances], precision, device)


class Server:
    """Toy-fit server with continuous batching (include/mipwa.h, mipwa_server_*)."""

    def __init__(self, precision=MIXED, device=0, hbm_budget_bytes=0):
        self._lib = L.load()
        h = C.c_void_p()
        rc = self._lib.mipwa_server_create(int(device), int(precision), int(hbm_budget_bytes), C.byref(h))
        if rc != 0:
            raise MipwaError(rc, "mipwa_server_create")
        self._h = h
        self._models = {}
        self._borrowed = {}  # job id -> the event arrays the server reads until the job's final result

    def _check(self, rc, what, ok=(0,)):
        if rc not in ok:
            raise MipwaError(rc, f"{what}: {self._lib.mipwa_server_last_error(self._h).decode()}")
        return rc

    def set_norm(self, s12, s13, w):
        s12, s13 = _f64(s12), _f64(s13)
        w = _f64(np.broadcast_to(w, s12.shape))
        self._check(self._lib.mipwa_server_set_norm(self._h, L.dptr(s12), L.dptr(s13), L.dptr(w), len(s12)), "set_norm")

    def submit(self, decay, knots, resonances, s12, s13, theta0, fixed=None, tol_edm=1e-4, max_iter=1000,
               hessian=False, copy=True):
        """Queue a fit.  copy=False lends the event arrays to the server instead of copying them
        (mipwa_server_submit_borrowed): they are held here until the job's final result is read."""
        mh = _ModelHolder(decay.M, decay.m1, decay.m2, decay.m3, decay.rD, knots,
                          [Resonance(r.spin, r.mass, r.width, r.radius) for r in resonances])
        s12, s13, th = _f64(s12), _f64(s13), _f64(theta0)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        opts = L.FitOptsC(float(tol_edm), int(max_iter), int(bool(hessian)))
        jid = C.c_longlong()
        fn = self._lib.mipwa_server_submit if copy else self._lib.mipwa_server_submit_borrowed
        self._check(fn(self._h, C.byref(mh.c), L.dptr(s12), L.dptr(s13), len(s12), L.dptr(th),
                       None if fx is None else fx.ctypes.data_as(C.POINTER(C.c_ubyte)), C.byref(opts),
                       C.byref(jid)), "submit")
        self._models[jid.value] = len(th)
        if not copy:
            self._borrowed[jid.value] = (s12, s13)
        return jid.value

    def _result(self, fn, jid, *extra):
        P = self._models[jid]
        th = np.empty(P)
        info = L.FitInfoC()
        lat = C.c_double()
        rc = fn(self._h, jid, *extra, L.dptr(th), C.byref(info), C.byref(lat))
        if rc == -8:
            return None
        self._borrowed.pop(jid, None)  # final: the server no longer reads the job's events
        self._check(rc, "result", ok=(0, -6, -7))
        if rc == -7:
            return {"status": rc}
        return {"status": rc, "theta": th, "nll": info.nll, "edm": info.edm, "n_iter": info.n_iter,
                "n_eval": info.n_eval, "latency_s": lat.value}

    def poll(self, jid):
        return self._result(self._lib.mipwa_server_poll, jid)

    def wait(self, jid, timeout_s=0.0):
        return self._result(self._lib.mipwa_server_wait, jid, C.c_double(timeout_s))

    def cancel(self, jid):
        self._check(self._lib.mipwa_server_cancel(self._h, jid), "cancel")

    def stats(self):
        st = L.ServeStatsC()
        self._check(self._lib.mipwa_server_stats(self._h, C.byref(st)), "stats")
        return {k: getattr(st, k) for k, _ in L.ServeStatsC._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mipwa_server_destroy(self._h)
            self._h = None
            self._borrowed = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
