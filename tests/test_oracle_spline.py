"""Pins for the oracle's natural cubic spline (Sec. 2: cubic spline through complex knots)."""
import json
import os

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import spline as sp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_worked_example_three_knots():
    g = _golden("spline_worked_examples.json")["three_knots"]
    kn = np.array(g["knots"])
    z = np.array(g["values"], dtype=complex)
    M = sp.second_derivatives(kn, z)
    assert M[1].real == pytest.approx(g["M1"], abs=1e-14)
    for s, want in g["S"]:
        assert sp.evaluate(kn, z, M, np.array([s]))[0].real == pytest.approx(want, abs=1e-14)


def test_worked_example_complex_plane_reading():
    """Re/Im splined separately (not magnitude and phase): the two readings differ at s = 1.5."""
    g = _golden("spline_worked_examples.json")["rotating_phase"]
    kn = np.array(g["knots"])
    a, phi = np.array(g["a"]), np.array(g["phi"])
    z = a * np.exp(1j * phi)
    M = sp.second_derivatives(kn, z)
    v = sp.evaluate(kn, z, M, np.array([g["s"]]))[0]
    assert v.real == pytest.approx(g["S_re"], abs=1e-12)
    assert v.imag == pytest.approx(g["S_im"], abs=1e-12)
    assert abs(v - complex(*g["magnitude_phase_reading"])) > 0.05


def test_matches_scipy_natural_spline(rng):
    for n in (3, 5, 20, 50):
        kn = np.sort(rng.uniform(0, 3, n))
        kn = np.unique(kn)
        z = rng.normal(size=len(kn)) + 1j * rng.normal(size=len(kn))
        s = rng.uniform(kn[0], kn[-1], 1000)
        M = sp.second_derivatives(kn, z)
        got = sp.evaluate(kn, z, M, s)
        ref = CubicSpline(kn, z.real, bc_type="natural")(s) + 1j * CubicSpline(kn, z.imag, bc_type="natural")(s)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(z).max())


def test_interpolates_knots_and_natural_ends(rng):
    kn = np.linspace(0.08, 2.99, 30)
    z = rng.normal(size=30) + 1j * rng.normal(size=30)
    M = sp.second_derivatives(kn, z)
    np.testing.assert_allclose(sp.evaluate(kn, z, M, kn), z, atol=1e-12)
    assert M[0] == 0 and M[-1] == 0
    # second derivative is continuous: it is linear in each interval and equals M at the knots
    ref = CubicSpline(kn, z.real, bc_type="natural")
    np.testing.assert_allclose(ref(kn, 2), M.real, atol=1e-8 * np.abs(M).max())


def test_linear_and_constant_data_exact(rng):
    kn = np.sort(rng.uniform(0, 3, 12))
    for z in (np.full(12, 1.3 - 0.4j), 0.7 * kn + 1j * (2 - kn)):
        M = sp.second_derivatives(kn, z)
        np.testing.assert_allclose(M, 0, atol=1e-12)
        s = rng.uniform(kn[0], kn[-1], 200)
        want = np.interp(s, kn, z.real) + 1j * np.interp(s, kn, z.imag)
        np.testing.assert_allclose(sp.evaluate(kn, z, M, s), want, atol=1e-12)


def test_interval_rule_and_extrapolation():
    kn = np.array([0.0, 1.0, 2.0, 4.0])
    j, t, _ = sp.locate(kn, np.array([0.0, 1.0, 1.5, 4.0, -0.1, 4.2]))
    assert list(j) == [0, 1, 1, 2, 0, 2]
    np.testing.assert_allclose(t, [0, 0, 0.5, 1.0, -0.1, 1.1])


def test_basis_adjoint_is_sum_of_cardinal_splines(rng):
    """sum_p g_p dS(s_p)/dz_k, brute force: spline through the unit vector e_k evaluated at s_p."""
    kn = np.sort(rng.uniform(0, 3, 9))
    s = rng.uniform(kn[0] - 0.01, kn[-1] + 0.01, 300)
    g = rng.normal(size=300) + 1j * rng.normal(size=300)
    got = sp.basis_adjoint(kn, s, g)
    want = np.zeros(9, dtype=complex)
    for k in range(9):
        e = np.zeros(9)
        e[k] = 1.0
        want[k] = np.sum(g * sp.evaluate(kn, e, sp.second_derivatives(kn, e), s))
    np.testing.assert_allclose(got, want, atol=1e-11)
