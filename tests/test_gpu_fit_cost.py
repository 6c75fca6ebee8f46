"""Mixed-precision fits cost about what FP64 fits cost (Sec. 2: the unbinned maximum-likelihood fit).

A 1M-event toy (D+ -> pi-pi+pi+, 30 knots, rho(770) + f2(1270)) against 1M uniform normalisation
points is fitted from one start in FP64 and in mixed precision, with the normalisation as a point sweep,
as the quadratic form, and by a serving job.  The mixed fit must land within 0.01 sigma of the FP64 fit
and take no more than 10 % (plus a few) more evaluations: rounding in the working precision must
neither move the minimum nor slow the minimiser down (its line search tolerates a relative noise of
1e-8 in -2 ln L, far above what FP32 streams with FP64 sums leave at this size).
"""
import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_KNOTS = 30
N_EVENTS = 1_000_000
N_NORM = 1_000_000


@pytest.fixture(scope="module")
def sample():
    from paper_1703_03284_amd import FP64, context_for
    wl = synth.C1
    d = wl.decay
    kn = synth.uniform_knots(d, N_KNOTS)
    truth = synth.truth_theta(N_KNOTS, wl.resonances, 71)
    gen = context_for(d, kn, wl.resonances, FP64)
    s12, s13, _ = gen.toy(truth, N_EVENTS, 72, n_probe=200_000)
    gen.close()
    n12, n13 = synth.uniform_phase_space(d, N_NORM, 73)
    w = np.full(N_NORM, synth.region_area_mc(d, 1 << 22, 5) / N_NORM)
    start = synth.perturb_theta(truth, N_KNOTS, wl.n_res, 74)
    return {"wl": wl, "knots": kn, "events": (s12, s13), "norm": (n12, n13, w), "start": start,
            "fixed": synth.fixed_mask(N_KNOTS, wl.n_res)}


def _context_fit(sample, precision, qform):
    from paper_1703_03284_amd import NORM_QFORM, context_for
    wl = sample["wl"]
    ctx = context_for(wl.decay, sample["knots"], wl.resonances, precision)
    if qform:
        ctx.set_norm_mode(NORM_QFORM)
    ctx.load_events(*sample["events"])
    ctx.load_norm(*sample["norm"])
    fit = ctx.fit(sample["start"], fixed=sample["fixed"], tol_edm=1e-4)
    ctx.close()
    return fit.theta, fit.sigma, fit.n_eval


def _serving_fit(sample, precision):
    from paper_1703_03284_amd import Server
    wl = sample["wl"]
    with Server(precision) as srv:
        srv.set_norm(*sample["norm"])
        r = srv.wait(srv.submit(wl.decay, sample["knots"], wl.resonances, *sample["events"], sample["start"],
                                fixed=sample["fixed"], tol_edm=1e-4))
    assert r["status"] == 0
    return r["theta"], r["n_eval"]


def _check(sample, th64, sig64, n64, thmx, nmx):
    free = np.flatnonzero(sample["fixed"] == 0)
    d = np.asarray(thmx) - np.asarray(th64)
    npair = N_KNOTS + sample["wl"].n_res
    d[1:2 * npair:2] = np.angle(np.exp(1j * d[1:2 * npair:2]))
    pull = (np.abs(d[free]) / sig64[free]).max()
    print(f"evaluations fp64 {n64}, mixed {nmx}; largest |d theta| / sigma {pull:.2e}")
    assert pull < 0.01
    assert nmx <= 1.1 * n64 + 5


@pytest.mark.parametrize("qform", [False, True], ids=["point_sweep", "quadratic_form"])
def test_mixed_context_fit_costs_as_much_as_fp64(sample, qform):
    from paper_1703_03284_amd import FP64, MIXED
    th64, sig64, n64 = _context_fit(sample, FP64, qform)
    thmx, _, nmx = _context_fit(sample, MIXED, qform)
    _check(sample, th64, sig64, n64, thmx, nmx)


def test_mixed_serving_fit_costs_as_much_as_fp64(sample):
    from paper_1703_03284_amd import FP64, MIXED
    # the FP64 context fit with the quadratic form gives the errors; serving fits in both precisions
    _, sig64, _ = _context_fit(sample, FP64, True)
    th64, n64 = _serving_fit(sample, FP64)
    thmx, nmx = _serving_fit(sample, MIXED)
    _check(sample, th64, sig64, n64, thmx, nmx)
