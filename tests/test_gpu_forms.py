"""The alternative S-wave forms through the C ABI: Cartesian knots and the isobar S-wave (Sec. 2),
against the oracle on the same inputs."""
import numpy as np
import pytest

import synth
from oracle import fit as OF
from oracle import forms as F
from oracle import generate as OG
from oracle import kinematics as K
from tests.cases import make_problem, rel

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-10, 1e-8), "mixed": (1e-6, 1e-4)}


def _prec(name):
    from paper_1703_03284_amd import FP64, MIXED
    return {"fp64": FP64, "mixed": MIXED}[name]


def _nll_ok(v, v_o, prec, scale=None):
    return rel(v, v_o) <= TOL[prec][0]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cartesian_knots_match_oracle(prec):
    from paper_1703_03284_amd import SWAVE_CARTESIAN
    wl = synth.C1
    prob = make_problem(wl, 3000, 20000, seed=41)
    N = wl.n_knots
    th = prob.theta.copy()
    a, p = th[0:2 * N:2].copy(), th[1:2 * N:2].copy()
    th[0:2 * N:2], th[1:2 * N:2] = a * np.cos(p), a * np.sin(p)
    ctx = prob.context(_prec(prec))
    ctx.set_swave_form(SWAVE_CARTESIAN)
    assert ctx.n_params == 2 * N + 4 * wl.n_res
    v, g = ctx.eval(th)
    v_o, g_o = F.cartesian_nll_and_grad(prob.model, th, prob.events, prob.oracle_norm(), shapes=False)
    assert _nll_ok(v, v_o, prec, prob.nll_scale()), (v, v_o)
    n_ck = 2 * N + 2 * wl.n_res
    assert np.abs(g[:n_ck] - g_o[:n_ck]).max() <= TOL[prec][1] * np.abs(g_o[:n_ck]).max()
    ctx.close()


def _isobar_problem(seed):
    wl = synth.ISO
    prob = make_problem(wl, 4000, 20000, seed=seed, eff="flat")
    th = synth.isobar_truth(wl.resonances, wl.seed("truth"))
    return wl, prob, th


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_isobar_swave_matches_oracle(prec):
    from paper_1703_03284_amd import SWAVE_ISOBAR
    wl, prob, th = _isobar_problem(42)
    ctx = prob.context(_prec(prec))
    ctx.set_swave_form(SWAVE_ISOBAR)
    R = wl.n_res
    assert ctx.n_params == 2 + 4 * R
    v, g = ctx.eval(th)
    v_o, g_o = F.isobar_nll_and_grad(prob.model, th, prob.events, prob.oracle_norm(), shapes=False)
    a = F.isobar_amplitude(prob.model, th, *prob.events)
    n12, n13, w = prob.oracle_norm()
    an = F.isobar_amplitude(prob.model, th, n12, n13)
    scale = 2 * np.abs(np.log(np.abs(a) ** 2)).sum() + 2 * len(a) * abs(np.log(np.sum(w * np.abs(an) ** 2)))
    assert _nll_ok(v, v_o, prec, scale), (v, v_o)
    n_c = 2 + 2 * R
    assert np.abs(g[:n_c] - g_o[:n_c]).max() <= TOL[prec][1] * np.abs(g_o[:n_c]).max()
    assert np.all(g[n_c:] == 0.0)
    ctx.close()


def test_isobar_scalar_mass_and_width_partials_on_the_fly():
    from paper_1703_03284_amd import SWAVE_ISOBAR
    wl, prob, th = _isobar_problem(43)
    ctx = prob.context(_prec("fp64"))
    ctx.set_swave_form(SWAVE_ISOBAR)
    ctx.set_fixed(synth.isobar_fixed(wl.n_res, float_shapes=True))
    v, g = ctx.eval(th)
    v_o, g_o = F.isobar_nll_and_grad(prob.model, th, prob.events, prob.oracle_norm(), shapes=True)
    assert rel(v, v_o) <= 1e-10
    assert np.abs(g - g_o).max() <= 1e-7 * np.abs(g_o).max()
    ctx.close()


def test_isobar_rejected_without_two_knots():
    from paper_1703_03284_amd import MipwaError, SWAVE_ISOBAR, context_for
    wl = synth.C1
    ctx = context_for(wl.decay, wl.knots(), wl.resonances)
    with pytest.raises(MipwaError):
        ctx.set_swave_form(SWAVE_ISOBAR)
    ctx.close()


@pytest.mark.slow
def test_isobar_fit_parity():
    """Same toy (drawn by the oracle's generator from the equivalent two-knot model), same start: the
    library's fit in the isobar form vs a scipy BFGS fit of the oracle's isobar likelihood."""
    from paper_1703_03284_amd import FP64, SWAVE_ISOBAR, context_for
    wl = synth.ISO
    R = wl.n_res
    prob = make_problem(wl, 10, 10, seed=0, eff="flat")
    truth = synth.isobar_truth(wl.resonances, wl.seed("truth"))
    spline_truth = np.concatenate([[truth[0] / 2, truth[1], truth[0] / 2, truth[1]], truth[2:]])
    s12, s13, _ = OG.toy(prob.model, spline_truth, 8000, seed=wl.seed("events"), n_probe=200_000)
    n12, n13 = synth.uniform_phase_space(wl.decay, 60_000, wl.seed("norm"))
    norm = (n12, n13, np.full(len(n12), K.area(prob.model) / len(n12)))
    fixed = synth.isobar_fixed(R)
    start = truth.copy()
    rng = np.random.Generator(np.random.PCG64(5))
    free = np.flatnonzero(fixed == 0)
    start[free[0::2]] *= rng.uniform(0.9, 1.1, len(free[0::2]))
    start[free[1::2]] += rng.uniform(-0.2, 0.2, len(free[1::2]))
    ref = OF.fit(prob.model, start, (s12, s13), norm, fixed, gtol=1e-6, objective=F.isobar_nll_and_grad,
                 n_pairs=1 + R)
    ctx = context_for(wl.decay, wl.knots(), wl.resonances, FP64)
    ctx.set_swave_form(SWAVE_ISOBAR)
    ctx.load_events(s12, s13)
    ctx.load_norm(*norm)
    res = ctx.fit(start, fixed=fixed, tol_edm=1e-8)
    d = res.theta - ref["theta"]
    d[1:2 + 2 * R:2] = np.angle(np.exp(1j * d[1:2 + 2 * R:2]))
    pulls = np.abs(d[free]) / ref["sigma"][free]
    assert pulls.max() < 0.01, pulls.max()
    assert np.abs(res.sigma[free] / ref["sigma"][free] - 1).max() < 0.01
    ctx.close()
