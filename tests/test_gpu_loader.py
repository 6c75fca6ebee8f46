"""Point loading on the device: validation order and messages, and independence from the order and
orientation in which the caller hands the points over.

The loader validates every point (region test, weight, efficiency), swaps each pair to s12 <= s13,
locates the spline cells and sorts stably by cell.  The first offending point is reported; a bad
point or weight comes before any bad efficiency.  Permuting the points or swapping the coordinates
of some of them changes only the order of the FP64 sums, so -2 ln L and the gradient agree to
rounding, and with the oracle to the usual FP64 bar.
"""
import numpy as np
import pytest

import synth
from tests.cases import make_problem, rel

pytestmark = pytest.mark.gpu


def _ctx(wl):
    from paper_1703_03284_amd import FP64, context_for
    return context_for(wl.decay, wl.knots(), wl.resonances, FP64)


def _raises(fn, status, text):
    from paper_1703_03284_amd import MipwaError
    with pytest.raises(MipwaError) as e:
        fn()
    assert e.value.status == status, e.value
    assert text in str(e.value), str(e.value)


def test_first_offending_point_is_reported():
    wl = synth.C1
    ctx = _ctx(wl)
    s12, s13 = synth.uniform_phase_space(wl.decay, 1000, 71)
    w = np.full(1000, 1e-3)
    eff = np.full(1000, 0.5)
    a, b = s12.copy(), s13.copy()
    a[7], a[3] = 0.01, np.nan               # outside, then non-finite earlier: index 3 is first
    _raises(lambda: ctx.load_events(a, b), -1, "point 3 ")
    a, b = s12.copy(), s13.copy()
    b[500] = 10.0
    _raises(lambda: ctx.load_events(a, b), -1, "point 500 ")
    # weights: a bad weight before a bad point is reported as the weight, and the other way round
    ww = w.copy()
    ww[3] = -1.0
    a = s12.copy()
    a[7] = 0.01
    _raises(lambda: ctx.load_norm(a, s13, ww), -1, "weight 3 ")
    ww = w.copy()
    ww[9] = np.inf
    _raises(lambda: ctx.load_norm(a, s13, ww), -1, "point 7 ")
    # efficiencies are checked once every point and weight is good
    e = eff.copy()
    e[4] = 0.0
    _raises(lambda: ctx.load_events(a, s13, eff=e), -1, "point 7 ")
    _raises(lambda: ctx.load_events(s12, s13, eff=e), -1, "efficiency 4 ")
    e[2] = np.nan
    _raises(lambda: ctx.load_norm(s12, s13, w, eff=e), -1, "efficiency 2 ")
    # a failed load leaves nothing half-loaded behind
    _raises(lambda: ctx.eval(wl.truth()), -4, "")
    ctx.close()


def test_order_and_orientation_of_the_input_do_not_matter():
    wl = synth.C2
    prob = make_problem(wl, 20000, 40000, seed=23)
    v_o, g_o = prob.oracle()
    base = prob.context(_fp64())
    v0, g0 = base.eval()
    base.close()
    rng = np.random.Generator(np.random.PCG64(5))
    pe, pn = rng.permutation(20000), rng.permutation(40000)
    swap = rng.random(20000) < 0.5
    e12, e13 = prob.events
    a = np.where(swap, e13, e12)[pe]
    b = np.where(swap, e12, e13)[pe]
    n12, n13, w = prob.norm
    from paper_1703_03284_amd import context_for
    ctx = context_for(wl.decay, prob.knots, wl.resonances, _fp64())
    ctx.load_events(a, b, eff=prob.eff_events[pe])       # the efficiency is symmetric
    ctx.load_norm(n13[pn], n12[pn], w[pn], eff=prob.eff_norm[pn])
    v, g = ctx.eval(prob.theta)
    ctx.close()
    assert rel(v, v0) <= 1e-12, (v, v0)
    assert np.abs(g - g0).max() <= 1e-10 * np.abs(g0).max()
    assert rel(v, v_o) <= 1e-10
    n_ck = 2 * wl.n_knots + 2 * wl.n_res
    assert np.abs(g[:n_ck] - g_o[:n_ck]).max() <= 1e-8 * np.abs(g_o[:n_ck]).max()


def test_reloading_replaces_the_points():
    """A second load of a different size replaces the first completely."""
    wl = synth.C1
    big = make_problem(wl, 5000, 30000, seed=31)
    small = make_problem(wl, 700, 9000, seed=32)
    ctx = big.context(_fp64())
    ctx.eval()
    ctx.load_events(*small.events, eff=small.eff_events)
    ctx.load_norm(*small.norm, eff=small.eff_norm)
    v, g = ctx.eval(small.theta)
    v_o, g_o = small.oracle()
    ctx.close()
    assert rel(v, v_o) <= 1e-10, (v, v_o)


def _fp64():
    from paper_1703_03284_amd import FP64
    return FP64


def test_region_tolerance_at_the_boundary():
    """Points within 1e-9 s_max of the Dalitz boundary are accepted (rounding of the caller's
    kinematics), points beyond it are rejected with the first offending index."""
    from oracle import kinematics as K
    from tests.conftest import oracle_model
    wl = synth.C1
    m = oracle_model(wl)
    tol = 1e-9 * K.smax(m)
    s12 = np.array([0.5, 1.0, 1.7, 2.2])
    lo, hi = K.s13_limits(m, s12)
    ctx = _ctx(wl)
    # just inside the tolerance band on both sides of the s13 range, and at the s12 ends
    a = np.concatenate([s12, s12, [K.smin(m) - 0.5 * tol]])
    b = np.concatenate([hi + 0.5 * tol, lo - 0.5 * tol, [K.s13_limits(m, np.array([K.smin(m)]))[0][0]]])
    ctx.load_events(a, b)
    # beyond the band: rejected
    b2 = b.copy()
    b2[2] = hi[2] + 3.0 * tol
    _raises(lambda: ctx.load_events(a, b2), -1, "point 2 ")
    a3 = a.copy()
    a3[-1] = K.smin(m) - 3.0 * tol
    _raises(lambda: ctx.load_events(a3, b), -1, "point 8 ")
    ctx.close()


def test_rejected_efficiency_table_leaves_the_previous_one():
    """A table that fails validation changes nothing: points loaded afterwards without per-point
    efficiencies still take the previous table, and the evaluation agrees with the oracle."""
    prob = make_problem(synth.C3, 3000, 8000, seed=41)
    ctx = prob.context(_fp64(), table_mode=True)
    v1, g1 = ctx.eval()
    bad = np.array(prob.table, dtype=np.float32)
    bad[3, 5] = 0.0
    d = synth.C3.decay
    _raises(lambda: ctx.set_eff_table(bad, d.smin, d.smax), -1, "positive")
    _raises(lambda: ctx.set_eff_table(bad[:1], d.smin, d.smax), -1, "nx, ny >= 2")
    ctx.load_events(*prob.events)
    ctx.load_norm(*prob.norm)
    v2, g2 = ctx.eval(prob.theta)
    ctx.close()
    assert v2 == v1 and np.array_equal(g2, g1)
    v_o, _ = prob.oracle()
    assert rel(v2, v_o) <= 1e-10, (v2, v_o)
