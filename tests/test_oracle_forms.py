"""Pins of the alternative S-wave forms of the oracle: Cartesian knots and the isobar S-wave (Sec. 2).

Cartesian: the same model as the polar form at the same knot values, with the polar gradient
recovered from the Cartesian one through the Jacobian of (a, phi) -> (Re z, Im z), and the gradient
against central differences.  Isobar: with no resonances A is a constant, so -2 ln L = 2 n ln(sum w)
whatever c_NR is; with resonances it equals the two-knot spline model carrying c_NR / 2 at both knots
(computed by the spline code, a different route); and its gradient, mass and width partials included,
against central differences.
"""
import numpy as np
import pytest

import synth
from oracle import Model
from oracle import forms as F
from oracle import kinematics as K
from oracle import likelihood as L
from tests.conftest import oracle_model


@pytest.fixture(scope="module")
def pts():
    wl = synth.C1
    ev = synth.uniform_phase_space(wl.decay, 1500, 61)
    s12, s13 = synth.uniform_phase_space(wl.decay, 8000, 62)
    m = oracle_model(wl)
    return ev, (s12, s13, np.full(len(s12), K.area(m) / len(s12)))


def _cartesian(theta, N):
    th = np.array(theta, copy=True)
    a, p = th[0:2 * N:2].copy(), th[1:2 * N:2].copy()
    th[0:2 * N:2], th[1:2 * N:2] = a * np.cos(p), a * np.sin(p)
    return th


def test_cartesian_is_the_polar_model_and_the_jacobian_links_the_gradients(pts):
    wl = synth.C1
    m = oracle_model(wl)
    N = wl.n_knots
    th = wl.start()
    ev, nm = pts
    v_p, g_p = L.nll_and_grad(m, th, ev, nm, shapes=False)
    v_c, g_c = F.cartesian_nll_and_grad(m, _cartesian(th, N), ev, nm, shapes=False)
    assert abs(v_c - v_p) <= 1e-12 * abs(v_p)
    a, p = th[0:2 * N:2], th[1:2 * N:2]
    gx, gy = g_c[0:2 * N:2], g_c[1:2 * N:2]
    np.testing.assert_allclose(gx * np.cos(p) + gy * np.sin(p), g_p[0:2 * N:2], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(a * (-gx * np.sin(p) + gy * np.cos(p)), g_p[1:2 * N:2], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(g_c[2 * N:], g_p[2 * N:], rtol=1e-12, atol=1e-12)


def test_cartesian_gradient_against_differences(pts):
    wl = synth.C1
    m = oracle_model(wl)
    th = _cartesian(wl.start(), wl.n_knots)
    ev, nm = pts
    _, g = F.cartesian_nll_and_grad(m, th, ev, nm, shapes=False)
    for p in (0, 1, 7, 2 * wl.n_knots - 1, 2 * wl.n_knots + 2):
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (F.cartesian_nll_and_grad(m, tp, ev, nm, shapes=False)[0]
              - F.cartesian_nll_and_grad(m, tm, ev, nm, shapes=False)[0]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-5 * max(1.0, abs(g[p])), (p, fd, g[p])


def test_isobar_without_resonances_is_normalised_away(pts):
    d = synth.C1.decay
    m = Model(d.M, d.m1, d.m2, d.m3, d.rD, (d.smin, d.smax), ())
    ev, nm = pts
    for c in ((1.0, 0.3), (0.2, -2.0), (5.0, 1.0)):
        v, g = F.isobar_nll_and_grad(m, np.array(c), ev, nm)
        assert abs(v - 2 * len(ev[0]) * np.log(nm[2].sum())) <= 1e-10 * abs(v)
        assert np.abs(g).max() <= 1e-9 * len(ev[0])


def test_isobar_equals_the_two_knot_spline_carrying_half_the_constant(pts):
    wl = synth.ISO
    m = oracle_model(wl)
    R = wl.n_res
    th = synth.isobar_truth(wl.resonances, wl.seed("truth"))
    th[0] = 1.3
    ev, nm = pts
    v_i, g_i = F.isobar_nll_and_grad(m, th, ev, nm, shapes=False)
    sp = np.concatenate([[th[0] / 2, th[1], th[0] / 2, th[1]], th[2:]])
    assert len(sp) == m.n_params
    v_s, g_s = L.nll_and_grad(m, sp, ev, nm, shapes=False)
    assert abs(v_i - v_s) <= 1e-12 * abs(v_s)
    assert abs(g_i[0] - 0.5 * (g_s[0] + g_s[2])) <= 1e-9 * max(1.0, abs(g_i[0]))
    assert abs(g_i[1] - (g_s[1] + g_s[3])) <= 1e-9 * max(1.0, abs(g_i[1]))
    np.testing.assert_allclose(g_i[2:2 + 2 * R], g_s[4:4 + 2 * R], rtol=1e-9, atol=1e-9)


def test_isobar_gradient_against_differences(pts):
    wl = synth.ISO
    m = oracle_model(wl)
    th = synth.isobar_truth(wl.resonances, wl.seed("truth"))
    ev, nm = pts
    _, g = F.isobar_nll_and_grad(m, th, ev, nm, shapes=True)
    R = wl.n_res
    for p in [0, 1, 4, 5] + list(range(2 + 2 * R, 2 + 4 * R)):
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (F.isobar_nll(m, tp, ev, nm) - F.isobar_nll(m, tm, ev, nm)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-5 * max(1.0, abs(g[p])), (p, fd, g[p])
