"""Three-body kinematics of D+ -> h- h+ h+ (test infrastructure only).

s12 and s13 are the invariant masses squared of (h1 h2) and (h1 h3) (Sec. 2, below Eq. 1); with
h1 the h- (Sec. 4: both axes are m^2(K+K-)), both are h+h- masses.  The allowed region is the
standard Dalitz region: for a given s12, s13 runs between
  (E1* + E3*)^2 - (p1* +/- p3*)^2,
with E1*, E3*, p1*, p3* the energies and momenta of h1 and h3 in the (12) rest frame.
"""
from __future__ import annotations

import warnings

import numpy as np
from scipy.integrate import IntegrationWarning, quad


def s13_limits(model, s12):
    """(s13_lo, s13_hi) at the given s12 (energy/momentum form in the (12) rest frame)."""
    s12 = np.asarray(s12, dtype=np.float64)
    rs = np.sqrt(s12)
    e1 = (s12 - model.m2 ** 2 + model.m1 ** 2) / (2.0 * rs)
    e3 = (model.M ** 2 - s12 - model.m3 ** 2) / (2.0 * rs)
    p1 = np.sqrt(np.maximum(e1 * e1 - model.m1 ** 2, 0.0))
    p3 = np.sqrt(np.maximum(e3 * e3 - model.m3 ** 2, 0.0))
    return (e1 + e3) ** 2 - (p1 + p3) ** 2, (e1 + e3) ** 2 - (p1 - p3) ** 2


def smin(model) -> float:
    return (model.m1 + model.m2) ** 2


def smax(model) -> float:
    return (model.M - model.m3) ** 2


def s23(model, s12, s13):
    return model.M ** 2 + model.m1 ** 2 + model.m2 ** 2 + model.m3 ** 2 - s12 - s13


def inside(model, s12, s13):
    s12 = np.asarray(s12, dtype=np.float64)
    s13 = np.asarray(s13, dtype=np.float64)
    ok = (s12 >= smin(model)) & (s12 <= smax(model))
    lo, hi = s13_limits(model, np.clip(s12, smin(model), smax(model)))
    return ok & (s13 >= lo) & (s13 <= hi)


def area(model) -> float:
    """|D| = integral over s12 of (s13_hi - s13_lo), by adaptive quadrature."""
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", IntegrationWarning)
        val, _ = quad(lambda s: float(np.subtract(*s13_limits(model, s)[::-1])),
                      smin(model), smax(model), epsabs=1e-14, epsrel=1e-14, limit=400)
    return val
