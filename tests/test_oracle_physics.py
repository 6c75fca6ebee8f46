"""Pins for the oracle's kinematics and resonance amplitudes (Sec. 2 Breit-Wigners, Sec. 4 kinematics)."""
import json
import os

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import kinematics as K
from oracle import resonance as R
from tests.conftest import oracle_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def pipipi():
    return oracle_model(synth.C2)


def test_dalitz_area_matches_independent_region_test(pipipi):
    g = json.load(open(os.path.join(GOLDEN, "dalitz_area.json")))
    area = K.area(pipipi)
    assert area == pytest.approx(g["pipipi"], rel=1e-11)
    # independent polynomial region test, Monte Carlo over the bounding box (4 sigma)
    n = 1 << 22
    acc = synth.box_acceptance(synth.D_PIPIPI, n, seed=3)
    box = (synth.D_PIPIPI.smax - synth.D_PIPIPI.smin) ** 2
    sig = np.sqrt(acc * (1 - acc) / n) * box
    assert abs(acc * box - area) < 4 * sig
    assert acc == pytest.approx(g["pipipi_box_acceptance"], abs=4 * np.sqrt(acc * (1 - acc) / n))
    kkk = oracle_model(synth.Workload("kkk", 9, "fp64", 1, 1, 40, (synth.PHI1020,), "flat", decay=synth.D_KKK))
    assert K.area(kkk) == pytest.approx(g["kkk"], rel=1e-11)


def test_region_tests_agree(pipipi, rng):
    d = synth.D_PIPIPI
    s12 = rng.uniform(d.smin, d.smax, 200000)
    s13 = rng.uniform(d.smin, d.smax, 200000)
    assert np.array_equal(K.inside(pipipi, s12, s13), synth.inside_region(d, s12, s13))


def test_limits_collapse_at_the_ends(pipipi):
    for s in (K.smin(pipipi), K.smax(pipipi)):
        lo, hi = K.s13_limits(pipipi, s)
        assert hi - lo == pytest.approx(0.0, abs=1e-7)


def test_pole_values(pipipi):
    """At x = m_r^2: q = q_r, p = p_r, B = 1, Gamma(x) = Gamma_r, so the dynamical part is i/(m_r Gamma_r)."""
    g = json.load(open(os.path.join(GOLDEN, "bw_pole.json")))
    for res in pipipi.res:
        d = R.dynamical(pipipi, res, np.array([res.mass ** 2]))[0]
        assert abs(d) == pytest.approx(1.0 / (res.mass * res.width), rel=1e-13)
        assert np.angle(d) == pytest.approx(np.pi / 2, abs=1e-13)
        assert R.running_width(pipipi, res, np.array([res.mass ** 2]))[0] == pytest.approx(res.width, rel=1e-14)
    mags = [abs(R.dynamical(pipipi, r, np.array([r.mass ** 2]))[0]) for r in pipipi.res]
    np.testing.assert_allclose(mags, g["magnitudes_rho770_f2_rho1450"], rtol=1e-4)


def test_phase_motion_and_half_width(pipipi):
    """Phase rises through pi/2 at the pole; |1/D|^2 is half its pole value where m^2 - x = +-m Gamma(x)."""
    res = pipipi.res[0]
    x = np.linspace(0.3, 1.0, 2001)
    ph = np.unwrap(np.angle(R.dynamical(pipipi, res, x)))
    assert np.all(np.diff(ph) > 0)
    for sgn in (+1, -1):
        # solve m^2 - x = sgn * m Gamma(x) by bisection, then check |D|^2 = 2 (m Gamma(x))^2
        f = lambda xx: res.mass ** 2 - xx - sgn * res.mass * R.running_width(pipipi, res, np.array([xx]))[0]
        a, b = (0.3, res.mass ** 2) if sgn > 0 else (res.mass ** 2, 1.0)
        for _ in range(200):
            c = 0.5 * (a + b)
            if np.sign(f(c)) == np.sign(f(a)):
                a = c
            else:
                b = c
        gw = R.running_width(pipipi, res, np.array([a]))[0]
        den = res.mass ** 2 - a - 1j * res.mass * gw
        assert abs(den) ** 2 == pytest.approx(2 * (res.mass * gw) ** 2, rel=1e-9)


def test_threshold_power_law(pipipi):
    """With zero barrier radius, Gamma(x) sqrt(x) / q^(2L+1) does not depend on x."""
    for spin in (1, 2):
        r0 = type(pipipi.res[0])(spin, 0.9, 0.1, 0.0)
        x = np.linspace(0.08, 2.5, 50)
        q = R.daughter_momentum(x, pipipi.m1, pipipi.m2)
        v = R.running_width(pipipi, r0, x) * np.sqrt(x) / q ** (2 * spin + 1)
        np.testing.assert_allclose(v, v[0], rtol=1e-12)


def test_momenta(pipipi, rng):
    x = rng.uniform(K.smin(pipipi) + 1e-3, K.smax(pipipi) - 1e-3, 100)
    q = R.daughter_momentum(x, pipipi.m1, pipipi.m2)
    # two daughters of mass m1, m2 with momentum q share the energy sqrt(x)
    np.testing.assert_allclose(np.sqrt(q ** 2 + pipipi.m1 ** 2) + np.sqrt(q ** 2 + pipipi.m2 ** 2), np.sqrt(x), rtol=1e-13)
    p = R.bachelor_momentum(x, pipipi.M, pipipi.m3)
    # in the resonance frame the mother moves with p: E_D - E_3 = sqrt(x)
    np.testing.assert_allclose(np.sqrt(p ** 2 + pipipi.M ** 2) - np.sqrt(p ** 2 + pipipi.m3 ** 2), np.sqrt(x), rtol=1e-12)
    # the s13 range is 4 p1* p3* = 4 q p at equal masses
    lo, hi = K.s13_limits(pipipi, x)
    np.testing.assert_allclose(hi - lo, 4 * q * p, rtol=1e-10)


def test_blatt_weisskopf(rng):
    q = rng.uniform(0.01, 1.0, 100)
    for L in (0, 1, 2):
        np.testing.assert_allclose(R.blatt_weisskopf(L, q, q, 1.5), 1.0)
    z = (1.5 * q) ** 2
    np.testing.assert_allclose(R.blatt_weisskopf(1, q, 0.3, 1.5) ** 2 * (1 + z), 1 + (1.5 * 0.3) ** 2, rtol=1e-13)


def test_zemach_orthogonality_and_boundary(pipipi):
    """At fixed x, T_1 and T_2 are Legendre P_1 and P_2 in the helicity angle: they integrate to zero
    over the s13 range, T_1 = +-(s13_hi - s13_lo) at the ends (+ at the lower end), and
    T_2 = (2/3)(s13_hi - s13_lo)^2 there."""
    for x in (0.2, 0.6, 1.2, 2.0, 2.8):
        lo, hi = K.s13_limits(pipipi, x)
        for L in (1, 2):
            val, _ = quad(lambda y: float(R.zemach(pipipi, L, np.array([x]), np.array([y]))[0]), lo, hi,
                          epsabs=1e-13)
            assert abs(val) < 1e-11 * (hi - lo) ** (L + 1)
        d = hi - lo
        t1 = R.zemach(pipipi, 1, np.array([x, x]), np.array([lo, hi]))
        np.testing.assert_allclose(t1, [d, -d], rtol=1e-9)
        t2 = R.zemach(pipipi, 2, np.array([x, x]), np.array([lo, hi]))
        np.testing.assert_allclose(t2, [2 * d * d / 3] * 2, rtol=1e-9)


def test_symmetrisation_is_exact(pipipi, rng):
    d = synth.D_PIPIPI
    s12, s13 = synth.uniform_phase_space(d, 1000, 11)
    for res in pipipi.res:
        a = R.symmetrised(pipipi, res, s12, s13)
        b = R.symmetrised(pipipi, res, s13, s12)
        assert np.array_equal(a, b)


def _case_model(base, case):
    from oracle import Model, Res
    return Model(base.M, base.m1, base.m2, base.m3, case["rD"], base.knots,
                 (Res(case["spin"], case["mass"], case["width"], case["radius"]),))


def _offpole_cases():
    return json.load(open(os.path.join(GOLDEN, "bw_offpole.json")))["cases"]


def test_offpole_hand_values(pipipi):
    """Off the pole each factor of the dynamical part differs from 1, so the hand-worked values pin
    which momentum enters which barrier factor with which radius (Sec. 2 Breit-Wigner)."""
    for c in _offpole_cases():
        m = _case_model(pipipi, c)
        res = m.res[0]
        x = np.array([c["x"]])
        assert R.daughter_momentum(x, m.m1, m.m2)[0] == pytest.approx(c["q"], rel=1e-13)
        assert R.bachelor_momentum(x, m.M, m.m3)[0] == pytest.approx(c["p"], rel=1e-13)
        assert R.blatt_weisskopf(res.spin, x * 0 + c["q"], c["q_r"], res.radius)[0] == pytest.approx(c["B_q"], rel=1e-13)
        assert R.blatt_weisskopf(res.spin, x * 0 + c["p"], c["p_r"], m.rD)[0] == pytest.approx(c["B_p"], rel=1e-13)
        assert R.running_width(m, res, x)[0] == pytest.approx(c["running_width"], rel=1e-12)
        d = R.dynamical(m, res, x)[0]
        assert d.real == pytest.approx(c["re"], rel=1e-12)
        assert d.imag == pytest.approx(c["im"], rel=1e-12)


def test_textbook_rbw_reduction(pipipi):
    """With L = 0 and both barrier radii zero the dynamical part is the textbook relativistic
    Breit-Wigner in the mass m = sqrt(x): 1 / (m_r^2 - m^2 - i m_r Gamma_r (q/q_r)(m_r/m)), with the
    pion momentum q = sqrt(m^2/4 - m_pi^2); checked at points away from the pole on both sides."""
    from oracle import Model, Res
    mr, gr = 0.990, 0.060
    m = Model(pipipi.M, pipipi.m1, pipipi.m2, pipipi.m3, 0.0, pipipi.knots, (Res(0, mr, gr, 0.0),))
    mass = np.linspace(0.3, 1.7, 57)
    qq = np.sqrt(mass ** 2 / 4 - pipipi.m1 ** 2)
    q0 = np.sqrt(mr ** 2 / 4 - pipipi.m1 ** 2)
    textbook = 1.0 / (mr ** 2 - mass ** 2 - 1j * mr * gr * (qq / q0) * (mr / mass))
    got = R.dynamical(m, m.res[0], mass ** 2)
    np.testing.assert_allclose(got.real, textbook.real, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got.imag, textbook.imag, rtol=1e-12, atol=1e-14)
    c = _offpole_cases()[2]
    d = R.dynamical(m, m.res[0], np.array([c["x"]]))[0]
    assert (d.real, d.imag) == (pytest.approx(c["re"], rel=1e-12), pytest.approx(c["im"], rel=1e-12))


def _planted(kind):
    """The dynamical part with one plausible mistake planted (test of the pins above)."""
    def dyn(model, res, x):
        q = R.daughter_momentum(x, model.m1, model.m2)
        q_r = R.daughter_momentum(res.mass ** 2, model.m1, model.m2)
        p = R.bachelor_momentum(x, model.M, model.m3)
        p_r = R.bachelor_momentum(res.mass ** 2, model.M, model.m3)
        rr, rd = (model.rD, res.radius) if kind == "radii swapped" else (res.radius, model.rD)
        bq = R.blatt_weisskopf(res.spin, q, q_r, rr)
        if kind == "no D factor":
            bp = 1.0
        elif kind == "q for p":
            bp = R.blatt_weisskopf(res.spin, q, q_r, rd)
        else:
            bp = R.blatt_weisskopf(res.spin, p, p_r, rd)
        gam = res.width * (q / q_r) ** (2 * res.spin + 1) * (res.mass / np.sqrt(x)) * bq * bq
        return bq * bp / (res.mass ** 2 - x - 1j * res.mass * gam)
    return dyn


@pytest.mark.parametrize("kind", ["radii swapped", "no D factor", "q for p"])
def test_offpole_pins_reject_planted_mistakes(pipipi, kind):
    """Each planted mistake moves an off-pole hand value by more than 1%; at the pole all of them
    agree with the correct form (which is why the pole pin alone could not see them)."""
    dyn = _planted(kind)
    worst = 0.0
    for c in _offpole_cases()[:2]:
        m = _case_model(pipipi, c)
        d = dyn(m, m.res[0], np.array([c["x"]]))[0]
        worst = max(worst, abs(d - complex(c["re"], c["im"])) / abs(complex(c["re"], c["im"])))
        pole = dyn(m, m.res[0], np.array([c["mass"] ** 2]))[0]
        assert abs(pole - 1j / (c["mass"] * c["width"])) < 1e-9 * abs(pole)
    assert worst > 1e-2
