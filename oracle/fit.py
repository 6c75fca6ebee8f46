"""Maximum-likelihood fit of the MIPWA model (test infrastructure only).

Sec. 2: the knot parameters {a_k, phi_k} and the resonance coefficients are determined by an
unbinned maximum-likelihood fit; interpolation correlates the parameters and makes the problem
non-linear.  The paper names no minimiser.  Reading taken: quasi-Newton BFGS on -2 ln L over the
floated parameters (scipy's implementation), then the Hessian H by central differences of the
analytic gradient, covariance V = 2 H^-1 (the function is -2 ln L), and the estimated distance to
the minimum EDM = (1/2) g^T H^-1 g.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from .likelihood import nll_and_grad


def canonical(model, theta, n_pairs=None):
    """Fold each (magnitude, phase) pair to magnitude >= 0 and phase in (-pi, pi]: the first n_pairs
    pairs of theta (default: the N knots and R coefficients of the polar spline layout)."""
    th = np.array(theta, dtype=np.float64, copy=True)
    if n_pairs is None:
        n_pairs = model.n_knots + model.n_res
    for k in range(n_pairs):
        a, p = th[2 * k], th[2 * k + 1]
        if a < 0:
            a, p = -a, p + np.pi
        p = np.pi - np.mod(np.pi - p, 2 * np.pi)
        th[2 * k], th[2 * k + 1] = a, p
    return th


def hessian(func_grad, x, step_rel=1e-4):
    n = len(x)
    H = np.zeros((n, n))
    for i in range(n):
        h = step_rel * max(1.0, abs(x[i]))
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        H[:, i] = (func_grad(xp)[1] - func_grad(xm)[1]) / (2 * h)
    return 0.5 * (H + H.T)


def fit(model, theta0, events, norm, fixed, log_eps_sum=0.0, gtol=1e-5, maxiter=5000, objective=None,
        n_pairs=None):
    """objective(model, theta, events, norm, log_eps_sum, shapes) -> (-2 ln L, gradient), default the
    polar spline form; n_pairs leading (magnitude, phase) pairs precede the masses and widths."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    fixed = np.asarray(fixed, dtype=bool)
    free = np.flatnonzero(~fixed)
    objective = objective or nll_and_grad
    if n_pairs is None:
        n_pairs = model.n_knots + model.n_res
    shapes = bool((~fixed[2 * n_pairs:]).any())

    def fg(x):
        th = theta0.copy()
        th[free] = x
        v, g = objective(model, th, events, norm, log_eps_sum, shapes=shapes)
        return v, g[free]

    res = minimize(fg, theta0[free], jac=True, method="BFGS",
                   options={"gtol": gtol, "maxiter": maxiter})
    x = res.x
    v, g = fg(x)
    H = hessian(fg, x)
    Hinv = np.linalg.inv(H)
    V = 2.0 * Hinv
    th = theta0.copy()
    th[free] = x
    cov = np.zeros((len(theta0), len(theta0)))
    cov[np.ix_(free, free)] = V
    return {
        "theta": canonical(model, th, n_pairs),
        "theta_raw": th,
        "nll": v,
        "edm": 0.5 * float(g @ Hinv @ g),
        "cov": cov,
        "sigma": np.sqrt(np.maximum(np.diag(cov), 0.0)),
        "n_eval": int(res.nfev),
        "n_iter": int(res.nit),
        "success": bool(res.success),
    }
