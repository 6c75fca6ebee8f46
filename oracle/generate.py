"""Toy Monte Carlo by accept-reject on |A|^2 eps (test infrastructure only).

Sec. 4 tests the fit on toy samples generated from the Dalitz-plot PDF; the paper does not state
the method.  Reading taken: plain accept-reject.  Candidates are drawn uniformly in the bounding
box [smin, smax]^2 from the Philox stream (candidate i -> (u12, u13, v)), mapped as
s = smin + (smax - smin) u (one product, then one sum), kept if inside the Dalitz region, and
accepted when f = |A|^2 eps > v f_max.  The first n accepted candidates, in candidate order, are
the sample.  f_max is 1.5 times the largest f over the first n_probe inside-candidates of the key
seed + 1000; if any candidate then exceeds f_max, f_max is doubled and generation restarts.
"""
from __future__ import annotations

import numpy as np

from .kinematics import inside, smax, smin
from .likelihood import amplitude
from .philox import candidate_uniforms

BLOCK = 1 << 20


def candidates(model, seed, first, count):
    u12, u13, v = candidate_uniforms(seed, first, count)
    lo, span = smin(model), smax(model) - smin(model)
    return lo + span * u12, lo + span * u13, v


def density(model, theta, s12, s13, eff=None):
    a = amplitude(model, theta, s12, s13)
    f = a.real ** 2 + a.imag ** 2
    return f if eff is None else f * eff(s12, s13)


def density_max(model, theta, seed, n_probe, eff=None):
    """Largest f over the first n_probe inside-candidates of key `seed`."""
    best, seen, first = 0.0, 0, 0
    while seen < n_probe:
        s12, s13, _ = candidates(model, seed, first, BLOCK)
        ok = np.flatnonzero(inside(model, s12, s13))[: n_probe - seen]
        if len(ok):
            best = max(best, float(density(model, theta, s12[ok], s13[ok], eff).max()))
        seen += len(ok)
        first += BLOCK
    return best


def accept_reject(model, theta, n, seed, fmax, eff=None, max_candidates=1 << 40):
    """(s12, s13, exceeded, n_candidates_used): first n accepted in candidate order."""
    out12, out13, have, first, exceeded = [], [], 0, 0, False
    while have < n and first < max_candidates:
        s12, s13, v = candidates(model, seed, first, BLOCK)
        ok = inside(model, s12, s13)
        f = np.zeros(BLOCK)
        idx = np.flatnonzero(ok)
        f[idx] = density(model, theta, s12[idx], s13[idx], eff)
        exceeded |= bool((f > fmax).any())
        acc = np.flatnonzero(ok & (f > v * fmax))
        out12.append(s12[acc])
        out13.append(s13[acc])
        have += len(acc)
        first += BLOCK
    s12 = np.concatenate(out12)[:n].copy()
    s13 = np.concatenate(out13)[:n].copy()
    return s12, s13, exceeded


def toy(model, theta, n, seed, eff=None, n_probe=1_000_000):
    fmax = 1.5 * density_max(model, theta, seed + 1000, n_probe, eff)
    while True:
        s12, s13, exceeded = accept_reject(model, theta, n, seed, fmax, eff)
        if not exceeded:
            return s12, s13, fmax
        fmax *= 2.0
