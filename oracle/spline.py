"""Natural cubic spline through complex knot values (test infrastructure only).

Sec. 2: the S-wave A_0(s) takes the value a_k exp(i phi_k) at each of N boundary points s_k and is
a cubic spline in the complex plane in between.  Readings taken (the paper's spline reference is
not reproduced): the real and imaginary parts are splined separately through z_k = a_k exp(i phi_k);
the boundary conditions are natural (second derivative zero at both end knots).

With h_j = s_{j+1} - s_j and second derivatives M_k, the interior knots satisfy
  h_{k-1} M_{k-1} + 2 (h_{k-1} + h_k) M_k + h_k M_{k+1} = 6 [(z_{k+1} - z_k)/h_k - (z_k - z_{k-1})/h_{k-1}],
and on interval j, with t = (s - s_j)/h_j,
  S(s) = (1-t) z_j + t z_{j+1} + (h_j^2/6) [((1-t)^3 - (1-t)) M_j + (t^3 - t) M_{j+1}].
The interval is j = clamp(#{knots <= s} - 1, 0, N-2) (a point exactly on a knot belongs to the
interval above it); t is not clamped, so points marginally outside the knot range use the end
cubic.
"""
from __future__ import annotations

import numpy as np


def system(knots):
    """(T, D) with T M = D z: row 0 and row N-1 fix M = 0, interior rows are the continuity equations."""
    s = np.asarray(knots, dtype=np.float64)
    n = len(s)
    h = np.diff(s)
    T = np.zeros((n, n))
    D = np.zeros((n, n))
    T[0, 0] = 1.0
    T[n - 1, n - 1] = 1.0
    for k in range(1, n - 1):
        T[k, k - 1] = h[k - 1]
        T[k, k] = 2.0 * (h[k - 1] + h[k])
        T[k, k + 1] = h[k]
        D[k, k - 1] = 6.0 / h[k - 1]
        D[k, k] = -6.0 / h[k] - 6.0 / h[k - 1]
        D[k, k + 1] = 6.0 / h[k]
    return T, D


def second_derivatives(knots, z):
    T, D = system(knots)
    return np.linalg.solve(T, D @ np.asarray(z))


def dM_dz(knots):
    """The real N x N matrix K with M = K z."""
    T, D = system(knots)
    return np.linalg.solve(T, D)


def locate(knots, s):
    """(j, t): interval index and unclamped local coordinate."""
    kn = np.asarray(knots, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    j = np.clip(np.searchsorted(kn, s, side="right") - 1, 0, len(kn) - 2)
    h = kn[j + 1] - kn[j]
    return j, (s - kn[j]) / h, h


def evaluate(knots, z, Mpp, s):
    j, t, h = locate(knots, s)
    u = 1.0 - t
    return (u * z[j] + t * z[j + 1]
            + (h * h / 6.0) * ((u ** 3 - u) * Mpp[j] + (t ** 3 - t) * Mpp[j + 1]))


def local_weights(knots, s):
    """Per point: j and the four real weights of (z_j, z_{j+1}, M_j, M_{j+1}) in S(s)."""
    j, t, h = locate(knots, s)
    u = 1.0 - t
    return j, u, t, (h * h / 6.0) * (u ** 3 - u), (h * h / 6.0) * (t ** 3 - t)


def basis_adjoint(knots, s, g):
    """sum_p g_p dS(s_p)/dz_k for all k (complex g, real basis), through M = K z."""
    n = len(knots)
    j, wa, wb, ma, mb = local_weights(knots, s)
    gz = (np.bincount(j, weights=(g * wa).real, minlength=n)
          + np.bincount(j + 1, weights=(g * wb).real, minlength=n)
          + 1j * (np.bincount(j, weights=(g * wa).imag, minlength=n)
                  + np.bincount(j + 1, weights=(g * wb).imag, minlength=n)))
    gm = (np.bincount(j, weights=(g * ma).real, minlength=n)
          + np.bincount(j + 1, weights=(g * mb).real, minlength=n)
          + 1j * (np.bincount(j, weights=(g * ma).imag, minlength=n)
                  + np.bincount(j + 1, weights=(g * mb).imag, minlength=n)))
    return gz + dM_dz(knots).T @ gm
