"""Fits by the library against the oracle's fit (Sec. 2: unbinned maximum-likelihood fit of the knot
values {a_k, phi_k} and the resonance coefficients; Sec. 4: fitted values judged against their errors).

One seeded toy of the small fit workload (D+ -> pi-pi+pi+, 10k events drawn by the oracle's
accept-reject at the truth, 100k uniform normalisation points, 20 knots, rho(770) + f2(1270)), one start.
The oracle fits it with scipy's BFGS and the covariance 2 H^-1; every library fit below starts from the
same point and must land within 0.01 sigma of the oracle's minimum in every floated parameter, with
errors within 1 % of the oracle's, and fit fractions within 0.01 of their own propagated error.
Covered: a context in FP64 and in mixed precision, with the normalisation as a point sweep and as the
quadratic form, and a serving job in each precision.
"""
import numpy as np
import pytest

import synth
from oracle import fit as OF
from oracle import generate as OG
from oracle import kinematics as K
from oracle import likelihood as L
from tests.conftest import oracle_model

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _fit_fractions(model, theta, norm):
    """Diagonal fit fractions FF_k (efficiency 1, the normalisation points' weights)."""
    return np.diag(L.fit_fractions(model, theta, L.integrals(model, theta, norm))).copy()


@pytest.fixture(scope="module")
def small_fit():
    wl = synth.C1
    m = oracle_model(wl)
    s12, s13, _ = OG.toy(m, wl.truth(), wl.n_events, seed=wl.seed("events"), n_probe=200_000)
    n12, n13 = synth.uniform_phase_space(wl.decay, wl.n_norm, wl.seed("norm"))
    norm = (n12, n13, np.full(len(n12), K.area(m) / len(n12)))
    ref = OF.fit(m, wl.start(), (s12, s13), norm, wl.fixed(), gtol=1e-6)
    free = np.flatnonzero(wl.fixed() == 0)
    # errors of the fit fractions: J V J^T with J from central differences of the oracle's fractions
    th = ref["theta_raw"]
    ff = _fit_fractions(m, th, norm)
    J = np.zeros((len(ff), len(th)))
    for p in free:
        h = 1e-6 * max(1.0, abs(th[p]))
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        J[:, p] = (_fit_fractions(m, tp, norm) - _fit_fractions(m, tm, norm)) / (2 * h)
    sigma_ff = np.sqrt(np.diag(J @ ref["cov"] @ J.T))
    return {"wl": wl, "model": m, "events": (s12, s13), "norm": norm, "ref": ref, "free": free,
            "ff": ff, "sigma_ff": sigma_ff}


def _pulls(sf, theta):
    wl, ref, free = sf["wl"], sf["ref"], sf["free"]
    d = np.asarray(theta) - ref["theta"]
    npair = wl.n_knots + wl.n_res
    d[1:2 * npair:2] = np.angle(np.exp(1j * d[1:2 * npair:2]))
    return np.abs(d[free]) / ref["sigma"][free]


def _prec(name):
    from paper_1703_03284_amd import FP64, MIXED
    return {"fp64": FP64, "mixed": MIXED}[name]


@pytest.mark.parametrize("prec,qform", [("fp64", False), ("mixed", False), ("mixed", True), ("fp64", True)],
                         ids=["fp64-points", "mixed-points", "mixed-qform", "fp64-qform"])
def test_context_fit_matches_oracle_fit(small_fit, prec, qform):
    from paper_1703_03284_amd import NORM_QFORM, context_for
    sf = small_fit
    wl = sf["wl"]
    ctx = context_for(wl.decay, wl.knots(), wl.resonances, _prec(prec))
    if qform:
        ctx.set_norm_mode(NORM_QFORM)
    ctx.load_events(*sf["events"])
    ctx.load_norm(*sf["norm"])
    res = ctx.fit(wl.start(), fixed=wl.fixed(), tol_edm=1e-8)
    pulls = _pulls(sf, res.theta)
    free = sf["free"]
    sig_ratio = res.sigma[free] / sf["ref"]["sigma"][free]
    ff = np.diag(ctx.fit_fractions(res.theta))
    ctx.close()
    print(f"{prec} qform={qform}: max |dtheta|/sigma {pulls.max():.2e}, sigma ratio "
          f"[{sig_ratio.min():.4f}, {sig_ratio.max():.4f}], max |dFF|/sigma_FF "
          f"{np.max(np.abs(ff - sf['ff']) / sf['sigma_ff']):.2e}")
    assert pulls.max() < 0.01, pulls.max()
    assert np.abs(sig_ratio - 1).max() < 0.01, sig_ratio
    assert np.all(np.abs(ff - sf["ff"]) < 0.01 * sf["sigma_ff"]), (ff, sf["ff"], sf["sigma_ff"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_serving_job_matches_oracle_fit(small_fit, prec):
    from paper_1703_03284_amd import Server
    sf = small_fit
    wl = sf["wl"]
    srv = Server(_prec(prec))
    srv.set_norm(*sf["norm"])
    j = srv.submit(wl.decay, wl.knots(), wl.resonances, *sf["events"], wl.start(), fixed=wl.fixed(), tol_edm=1e-8)
    r = srv.wait(j)
    srv.close()
    assert r["status"] == 0, r
    pulls = _pulls(sf, r["theta"])
    print(f"serving {prec}: max |dtheta|/sigma {pulls.max():.2e}")
    assert pulls.max() < 0.01, pulls.max()


def test_mixed_gradient_error_weighted_by_sigma(small_fit):
    """The mixed-precision gradient error, weighted by the oracle's errors, stays below 1e-4 in every
    floated parameter: since the shift of the minimum is V dg, a bound of 1e-4 on |dg_p| sigma_p keeps
    it under 0.01 sigma for up to ~100 correlated parameters.  Checked at the start point and at the
    oracle's minimum (where the gradient itself is ~0 and only the error remains)."""
    from paper_1703_03284_amd import MIXED, context_for
    sf = small_fit
    wl, m, free = sf["wl"], sf["model"], sf["free"]
    sig = sf["ref"]["sigma"]
    ctx = context_for(wl.decay, wl.knots(), wl.resonances, MIXED)
    ctx.load_events(*sf["events"])
    ctx.load_norm(*sf["norm"])
    for th in (wl.start(), sf["ref"]["theta_raw"]):
        v, g = ctx.eval(th)
        v_o, g_o = L.nll_and_grad(m, th, sf["events"], sf["norm"], shapes=False)
        weighted = np.abs(g[free] - g_o[free]) * sig[free]
        print(f"|d(-2lnL)| {abs(v - v_o):.3e} (rel {abs(v - v_o) / abs(v_o):.2e}), "
              f"max |dg| sigma {weighted.max():.2e}")
        assert abs(v - v_o) <= 1e-6 * abs(v_o)
        assert weighted.max() <= 1e-4, weighted.max()
    ctx.close()
