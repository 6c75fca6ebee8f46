"""The oracle over large point sets, split into chunks across worker processes (test infrastructure
only: the full-size checks and the benchmark's CPU baseline use it).

Nothing here changes what the oracle computes.  The sums of likelihood.point_sums (and the component
integrals) over disjoint chunks of the points add up to the sums over all of them; the chunks are
combined in a fixed order, so the result does not depend on the number of workers beyond the
rounding of that order.  The point arrays are written once to .npy files that the workers map
read-only; workers are started with the "spawn" method, so they share no state (and no GPU context)
with the parent.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import shutil
import tempfile

import numpy as np

from . import likelihood as L

_W = {}


def _init(spec):
    from threadpoolctl import threadpool_limits
    _W["limits"] = threadpool_limits(limits=1)
    _W["model"] = spec["model"]
    for key, path in spec["arrays"].items():
        _W[key] = np.load(path, mmap_mode="r")


def _task(args):
    kind, lo, hi, theta, shapes = args
    m = _W["model"]
    if kind == "data":
        return L.point_sums(m, theta, np.asarray(_W["e12"][lo:hi]), np.asarray(_W["e13"][lo:hi]), None, shapes)
    if kind == "norm":
        return L.point_sums(m, theta, np.asarray(_W["n12"][lo:hi]), np.asarray(_W["n13"][lo:hi]),
                            np.asarray(_W["nw"][lo:hi]), shapes)
    if kind == "integrals":
        return L.integrals(m, theta, (np.asarray(_W["n12"][lo:hi]), np.asarray(_W["n13"][lo:hi]),
                                      np.asarray(_W["nw0"][lo:hi])))
    if kind == "info":
        free = shapes
        return _info_sums(m, theta, free, np.asarray(_W["n12"][lo:hi]), np.asarray(_W["n13"][lo:hi]),
                          np.asarray(_W["nw"][lo:hi]))
    raise ValueError(kind)


def _info_sums(model, theta, free, s12, s13, w):
    """Weighted sums for the expected information per event, Cov_P(grad ln|A|^2) with P proportional
    to w |A|^2 over the points: (sum p, sum p G, sum p G G^T) with G the per-point central differences
    of ln|A|^2 in each free parameter."""
    th = np.asarray(theta, dtype=np.float64)
    a = L.amplitude(model, th, s12, s13)
    p = w * (a.real ** 2 + a.imag ** 2)
    G = np.empty((len(free), len(s12)))
    for i, k in enumerate(free):
        h = 1e-5 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        ap, am = L.amplitude(model, tp, s12, s13), L.amplitude(model, tm, s12, s13)
        G[i] = (np.log(ap.real ** 2 + ap.imag ** 2) - np.log(am.real ** 2 + am.imag ** 2)) / (2 * h)
    return float(p.sum()), G @ p, (G * p) @ G.T


class OraclePool:
    """events = (s12, s13); norm = (s12, s13, w) with w the weight times the efficiency; w_plain (default
    w) is the weight alone, for the component integrals with efficiency 1."""

    def __init__(self, model, events, norm, log_eps_sum=0.0, w_plain=None, workers=None, chunk=L.CHUNK):
        self.model = model
        self.n_events = len(events[0])
        self.n_norm = len(norm[0])
        self.log_eps_sum = float(log_eps_sum)
        self.chunk = int(chunk)
        self.workers = int(workers or min(16, len(os.sched_getaffinity(0))))
        self._dir = tempfile.mkdtemp(prefix="oracle_pool_")
        arrays = {"e12": events[0], "e13": events[1], "n12": norm[0], "n13": norm[1], "nw": norm[2],
                  "nw0": norm[2] if w_plain is None else w_plain}
        paths = {}
        for key, a in arrays.items():
            paths[key] = os.path.join(self._dir, key + ".npy")
            np.save(paths[key], np.ascontiguousarray(a, dtype=np.float64))
        self._pool = mp.get_context("spawn").Pool(self.workers, initializer=_init,
                                                  initargs=({"model": model, "arrays": paths},))

    def _ranges(self, n, chunk=None):
        c = chunk or self.chunk
        return [(lo, min(n, lo + c)) for lo in range(0, n, c)]

    @staticmethod
    def _add(parts):
        out = list(parts[0])
        for p in parts[1:]:
            out = [a + b for a, b in zip(out, p)]
        return tuple(out)

    def nll_and_grad(self, theta, shapes=False):
        th = np.asarray(theta, dtype=np.float64)
        tasks = [("data", lo, hi, th, shapes) for lo, hi in self._ranges(self.n_events)]
        nd = len(tasks)
        tasks += [("norm", lo, hi, th, shapes) for lo, hi in self._ranges(self.n_norm)]
        parts = self._pool.map(_task, tasks, chunksize=1)
        return L.combine(self.model, th, self.n_events, self._add(parts[:nd]), self._add(parts[nd:]),
                         self.log_eps_sum)

    def integrals(self, theta):
        """I_jk over the normalisation points with the plain weights (efficiency 1)."""
        th = np.asarray(theta, dtype=np.float64)
        parts = self._pool.map(_task, [("integrals", lo, hi, th, False) for lo, hi in self._ranges(self.n_norm)],
                               chunksize=1)
        return sum(parts[1:], parts[0])

    def expected_sigma(self, theta, free, n_sub):
        """Errors sqrt(diag(V)) with V the inverse of the expected information n Cov_P(grad ln|A|^2), from
        the first n_sub normalisation points weighted by w |A|^2 (the density of the events)."""
        th = np.asarray(theta, dtype=np.float64)
        free = np.asarray(free)
        n_sub = min(int(n_sub), self.n_norm)
        c = max(1, -(-n_sub // self.workers))
        parts = self._pool.map(_task, [("info", lo, hi, th, free) for lo, hi in self._ranges(n_sub, c)],
                               chunksize=1)
        sp, sg, sgg = self._add(parts)
        mean = sg / sp
        cov = sgg / sp - np.outer(mean, mean)
        V = np.linalg.inv(self.n_events * cov)
        sigma = np.zeros(len(th))
        sigma[free] = np.sqrt(np.diag(V))
        return sigma

    def close(self):
        if getattr(self, "_pool", None) is not None:
            self._pool.close()
            self._pool.join()
            self._pool = None
        if getattr(self, "_dir", None):
            shutil.rmtree(self._dir, ignore_errors=True)
            self._dir = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
