"""Pins for the oracle's amplitude sum, -2 ln L, gradient, integrals and fit fractions
(Sec. 2 Eq. 1 and the unbinned likelihood; Sec. 4 normalisation every iteration)."""
import numpy as np
import pytest
from scipy.integrate import dblquad

import synth
from oracle import kinematics as K
from oracle import likelihood as L
from oracle.model import Model, Res
from tests.conftest import oracle_model


def _small_problem(n_ev=400, n_norm=3000, workload=synth.C2, seed=5):
    m = oracle_model(workload)
    th = workload.start()
    ev = synth.uniform_phase_space(workload.decay, n_ev, seed)
    s12, s13 = synth.uniform_phase_space(workload.decay, n_norm, seed + 1)
    w = np.full(n_norm, K.area(m) / n_norm) * synth.PolyEfficiency.seeded(workload.decay, 4)(s12, s13)
    return m, th, ev, (s12, s13, w)


@pytest.fixture(scope="module")
def small():
    return _small_problem()


def test_global_phase_and_scale_invariance(small):
    m, th, ev, nm = small
    base = L.nll(m, th, ev, nm)
    N, R = m.n_knots, m.n_res
    t2 = th.copy()
    t2[1:2 * N:2] += 0.7
    t2[2 * N + 1:2 * N + 2 * R:2] += 0.7
    t2[0:2 * N:2] *= 1.9
    t2[2 * N:2 * N + 2 * R:2] *= 1.9
    assert L.nll(m, t2, ev, nm) == pytest.approx(base, rel=1e-13)


def test_knot_sign_twin(small):
    m, th, ev, nm = small
    t2 = th.copy()
    t2[6] = -t2[6]
    t2[7] += np.pi
    assert L.nll(m, t2, ev, nm) == pytest.approx(L.nll(m, th, ev, nm), rel=1e-13)


def test_swapping_event_coordinates_is_exact(small):
    m, th, (s12, s13), nm = small
    sw = np.arange(len(s12)) % 3 == 0
    a12, a13 = np.where(sw, s13, s12), np.where(sw, s12, s13)
    assert L.nll(m, th, (a12, a13), nm) == L.nll(m, th, (s12, s13), nm)


def test_constant_swave_normalisation():
    """All z_k = 1 and no resonances: A = 2 everywhere, so I = 4 sum_j w_j = 4 |D| for uniform weights."""
    w0 = synth.C1
    m = Model(w0.decay.M, w0.decay.m1, w0.decay.m2, w0.decay.m3, w0.decay.rD, tuple(w0.knots()), ())
    th = np.zeros(2 * m.n_knots)
    th[0::2] = 1.0
    s12, s13 = synth.uniform_phase_space(w0.decay, 5000, 3)
    area = K.area(m)
    I = L.norm_integral(m, th, (s12, s13, np.full(5000, area / 5000)))
    assert I == pytest.approx(4 * 5.063084362536, rel=1e-11)


def test_one_event_one_point_by_hand(small):
    m, th, _, _ = small
    x, y = (0.61, 1.42), (1.1, 0.95)
    ax = L.amplitude(m, th, np.array([x[0]]), np.array([x[1]]))[0]
    ay = L.amplitude(m, th, np.array([y[0]]), np.array([y[1]]))[0]
    w = 0.37
    want = -2 * np.log(abs(ax) ** 2) + 2 * np.log(w * abs(ay) ** 2)
    got = L.nll(m, th, (np.array([x[0]]), np.array([x[1]])), (np.array([y[0]]), np.array([y[1]]), np.array([w])))
    assert got == pytest.approx(want, rel=1e-14)


def test_mc_integral_agrees_with_quadrature():
    """Uniform-MC normalisation vs. adaptive 2D quadrature of |A|^2 over the Dalitz region (4 sigma)."""
    w0 = synth.C1
    m = oracle_model(w0, knots=synth.uniform_knots(w0.decay, 5))
    th = synth.truth_theta(5, w0.resonances, 77)
    area = K.area(m)
    n = 200_000
    s12, s13 = synth.uniform_phase_space(w0.decay, n, 21)
    a = L.amplitude(m, th, s12, s13)
    f = a.real ** 2 + a.imag ** 2
    mc, err = area * f.mean(), area * f.std() / np.sqrt(n)
    val, _ = dblquad(lambda y, x: float(abs(L.amplitude(m, th, np.array([x]), np.array([y]))[0]) ** 2),
                     K.smin(m), K.smax(m), lambda x: float(K.s13_limits(m, x)[0]),
                     lambda x: float(K.s13_limits(m, x)[1]), epsabs=1e-4, epsrel=1e-5)
    assert abs(mc - val) < 4 * err


def test_gradient_matches_central_differences(small):
    m, th, ev, nm = small
    v, g = L.nll_and_grad(m, th, ev, nm, shapes=True)
    assert v == pytest.approx(L.nll(m, th, ev, nm), rel=1e-14)
    h = 1e-6
    fd = np.zeros_like(g)
    for p in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd[p] = (L.nll(m, tp, ev, nm) - L.nll(m, tm, ev, nm)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=0, atol=2e-5 * np.abs(g).max())


def test_gradient_null_directions(small):
    """Global phase and global scale leave -2 ln L unchanged, so two gradient combinations vanish."""
    m, th, ev, nm = small
    _, g = L.nll_and_grad(m, th, ev, nm, shapes=False)
    N, R = m.n_knots, m.n_res
    phase = g[1:2 * N:2].sum() + g[2 * N + 1:2 * N + 2 * R:2].sum()
    scale = (th[0:2 * N:2] * g[0:2 * N:2]).sum() + (th[2 * N:2 * N + 2 * R:2] * g[2 * N:2 * N + 2 * R:2]).sum()
    assert abs(phase) < 1e-10 * np.abs(g).max()
    assert abs(scale) < 1e-10 * np.abs(g).max()


def test_integrals_and_fit_fractions(small):
    m, th, _, nm = small
    I = L.integrals(m, th, nm)
    c = L.coefficient_vector(m, th)
    np.testing.assert_allclose(I, I.conj().T, atol=1e-12 * np.abs(I).max())
    total = (np.outer(c, c.conj()) * I).sum()
    assert total.real == pytest.approx(L.norm_integral(m, th, nm), rel=1e-12)
    assert abs(total.imag) < 1e-12 * abs(total)
    ff = L.fit_fractions(m, th, I)
    assert ff.sum() == pytest.approx(1.0, abs=1e-14)
    # diagonal fraction of a resonance = direct sum of |c_r R_r|^2 over the points / I
    s12, s13, w = nm
    a0, rs, a = L.components(m, th, s12, s13)
    direct = np.sum(w * abs(c[2] * rs[1]) ** 2) / np.sum(w * abs(a) ** 2)
    assert ff[2, 2] == pytest.approx(direct, rel=1e-12)
    # single component: FF = 1
    th1 = th.copy()
    th1[2 * m.n_knots:2 * m.n_knots + 2 * m.n_res:2] = 0.0
    assert L.fit_fractions(m, th1, L.integrals(m, th1, nm))[0, 0] == pytest.approx(1.0, abs=1e-14)


def test_hist_lookup(rng):
    lo, hi, nb = 0.1, 2.9, 20
    d = (hi - lo) / nb
    c = lo + (np.arange(nb) + 0.5) * d
    tab = (0.3 + 0.2 * c[:, None] - 0.1 * c[None, :]).astype(np.float64)
    # exact at the centres; a linear function is reproduced between the outer centres
    i, j = rng.integers(0, nb, 50), rng.integers(0, nb, 50)
    np.testing.assert_allclose(L.hist_lookup(tab, lo, hi, c[i], c[j]), tab[i, j], atol=1e-14)
    s12, s13 = rng.uniform(c[0], c[-1], 500), rng.uniform(c[0], c[-1], 500)
    np.testing.assert_allclose(L.hist_lookup(tab, lo, hi, s12, s13), 0.3 + 0.2 * s12 - 0.1 * s13, atol=1e-13)
    # constant beyond the outermost centres
    np.testing.assert_allclose(L.hist_lookup(tab, lo, hi, np.array([lo]), np.array([hi])), tab[0, -1], atol=1e-14)
