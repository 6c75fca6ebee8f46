"""The normalisation integral as a quadratic form over per-cell moments (fixed shapes), against the
oracle's direct sum over the same normalisation points and against the library's point sweep."""
import numpy as np
import pytest

import synth
from tests.cases import make_problem, rel

pytestmark = pytest.mark.gpu


def _ctx(prob, prec):
    from paper_1703_03284_amd import FP64, MIXED, NORM_QFORM
    ctx = prob.context({"fp64": FP64, "mixed": MIXED}[prec])
    ctx.set_norm_mode(NORM_QFORM)
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("wl,seed", [(synth.C1, 51), (synth.C2, 52), (synth.KKK, 53)], ids=["C1", "C2", "KKK"])
def test_quadratic_form_matches_oracle(wl, seed, prec):
    prob = make_problem(wl, 3000, 20000, seed=seed)
    ctx = _ctx(prob, prec)
    v, g = ctx.eval()
    v_o, g_o = prob.oracle()
    n_ck = 2 * wl.n_knots + 2 * wl.n_res
    err = np.abs(g[:n_ck] - g_o[:n_ck])
    if prec == "fp64":
        assert rel(v, v_o) <= 1e-10, (v, v_o)
        assert err.max() <= 1e-8 * np.abs(g_o[:n_ck]).max()
    elif wl is not synth.KKK:
        assert rel(v, v_o) <= 1e-6, (v, v_o, rel(v, v_o))
        assert err.max() <= 1e-4 * np.abs(g_o[:n_ck]).max(), (err.max(), np.abs(g_o[:n_ck]).max())
    else:
        # K-K+K+ with phi(1020): -2 ln L and the phi coefficient's gradient cancel (data and
        # normalisation sums of ~1.7e4 to 245), and FP32 rounding of the inputs shared by all points is
        # coherent across the terms; an FP64 emulation of the FP32 inputs and data-side arithmetic
        # gives 5e-6 of their size.  Bounds relative to the size of the summed terms.
        assert abs(v - v_o) <= 1e-6 * prob.nll_scale(), (v, v_o)
        bound = 1e-4 * np.abs(g_o[:n_ck]).max() + 1e-5 * prob.grad_scale()[:n_ck]
        assert np.all(err <= bound), (np.argmax(err - bound), err.max())
    ctx.close()


def test_quadratic_form_equals_the_point_sweep_and_follows_new_shapes():
    from paper_1703_03284_amd import FP64, NORM_POINTS, NORM_QFORM
    wl = synth.C2
    prob = make_problem(wl, 4000, 30000, seed=54)
    ctx = prob.context(FP64)
    th = prob.theta.copy()
    vals = {}
    for mode in (NORM_POINTS, NORM_QFORM, NORM_POINTS):
        ctx.set_norm_mode(mode)
        vals.setdefault(mode, []).append(ctx.eval(th))
    (vp, gp), (vq, gq) = vals[NORM_POINTS][0], vals[NORM_QFORM][0]
    assert rel(vq, vp) <= 1e-12
    assert np.abs(gq - gp).max() <= 1e-10 * np.abs(gp).max()
    assert vals[NORM_POINTS][1][0] == vp
    # new fixed shapes: the resonance amplitudes and the moments are rebuilt
    ctx.set_norm_mode(NORM_QFORM)
    th2 = th.copy()
    th2[-3] += 0.01
    th2[-2] *= 1.04
    v2, _ = ctx.eval(th2)
    assert rel(v2, prob.oracle(theta=th2)[0]) <= 1e-10
    ctx.close()


def test_floated_shapes_fall_back_to_the_point_sweep():
    wl = synth.C4
    prob = make_problem(wl, 2000, 10000, seed=55)
    ctx = _ctx(prob, "fp64")
    ctx.set_fixed(wl.fixed())
    v, g = ctx.eval()
    v_o, g_o = prob.oracle(shapes=True)
    assert rel(v, v_o) <= 1e-10
    assert np.abs(g - g_o).max() <= 1e-7 * np.abs(g_o).max()
    ctx.close()


def test_fit_with_the_quadratic_form_matches_the_point_sweep_fit():
    from paper_1703_03284_amd import FP64, NORM_QFORM
    from oracle import generate as OG
    wl = synth.C1
    prob = make_problem(wl, 10, 30000, seed=56)
    s12, s13, _ = OG.toy(prob.model, wl.truth(), 6000, seed=57, n_probe=100_000)
    res = {}
    for q in (False, True):
        from paper_1703_03284_amd import context_for
        ctx = context_for(wl.decay, wl.knots(), wl.resonances, FP64)
        if q:
            ctx.set_norm_mode(NORM_QFORM)
        ctx.load_events(s12, s13)
        ctx.load_norm(*prob.norm)
        res[q] = ctx.fit(wl.start(), fixed=wl.fixed(), tol_edm=1e-8)
        ctx.close()
    free = np.flatnonzero(wl.fixed() == 0)
    d = res[True].theta - res[False].theta
    d[1::2] = np.angle(np.exp(1j * d[1::2]))
    assert (np.abs(d[free]) / res[False].sigma[free]).max() < 1e-3
