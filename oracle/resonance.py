"""P- and D-wave resonance amplitudes (test infrastructure only).

Sec. 2: a resonance with non-zero spin is a relativistic Breit-Wigner times a real spin-dependent
angular factor.  The paper's reference for the exact form is not reproduced; the reading taken is
the standard Dalitz-plot formalism for a resonance r in the (a b) channel with bachelor c:

  BW_r(x, y) = B_L(q, q_r; R_r) B_L(p, p_r; r_D) T_L(x, y) / (m_r^2 - x - i m_r Gamma_r(x))
  Gamma_r(x) = Gamma_r (q/q_r)^(2L+1) (m_r/sqrt(x)) B_L(q, q_r; R_r)^2

x is the (a b) invariant mass squared and y = m^2(a c); q is the daughter momentum in the resonance
rest frame, p the bachelor momentum in the same frame; q_r and p_r are their values at x = m_r^2.
Blatt-Weisskopf factors with z = (rho q)^2:  B_0 = 1,  B_1 = sqrt((1+z_r)/(1+z)),
B_2 = sqrt((z_r^2+3z_r+9)/(z^2+3z+9)).  Zemach angular factors:
  T_1 = m^2(bc) - m^2(ac) + (M^2 - m_c^2)(m_a^2 - m_b^2)/x
  T_2 = T_1^2 - (1/3)(x - 2M^2 - 2m_c^2 + (M^2-m_c^2)^2/x)(x - 2m_a^2 - 2m_b^2 + (m_a^2-m_b^2)^2/x)
Particle a is always the h- (particle 1) and b the h+ in the resonance.

Sec. 4: the two h+ are identical, so every amplitude is symmetrised over the two h+h- axes:
  R_r(s12, s13) = BW_r(s12, s13) + BW_r(s13, s12)     (no 1/sqrt(2): it cancels in the PDF).
"""
from __future__ import annotations

import numpy as np

from .kinematics import s23


def kallen(a, b, c):
    return a * a + b * b + c * c - 2.0 * (a * b + b * c + c * a)


def daughter_momentum(x, ma, mb):
    return np.sqrt(np.maximum(kallen(x, ma * ma, mb * mb), 0.0)) / (2.0 * np.sqrt(x))


def bachelor_momentum(x, M, mc):
    return np.sqrt(np.maximum(kallen(M * M, x, mc * mc), 0.0)) / (2.0 * np.sqrt(x))


def barrier_poly(L, z):
    if L == 0:
        return np.ones_like(z)
    if L == 1:
        return 1.0 + z
    if L == 2:
        return z * z + 3.0 * z + 9.0
    raise ValueError("spin must be 0, 1 or 2")


def blatt_weisskopf(L, q, q_r, radius):
    return np.sqrt(barrier_poly(L, (radius * q_r) ** 2) / barrier_poly(L, (radius * q) ** 2))


def zemach(model, L, x, y):
    """Angular factor for the resonance in the invariant x, with y the other h-h+ invariant."""
    M2, ma2, mb2, mc2 = model.M ** 2, model.m1 ** 2, model.m2 ** 2, model.m3 ** 2
    if L == 0:
        return np.ones_like(x)
    t1 = s23(model, x, y) - y + (M2 - mc2) * (ma2 - mb2) / x
    if L == 1:
        return t1
    if L == 2:
        return t1 * t1 - (x - 2.0 * M2 - 2.0 * mc2 + (M2 - mc2) ** 2 / x) * \
            (x - 2.0 * ma2 - 2.0 * mb2 + (ma2 - mb2) ** 2 / x) / 3.0
    raise ValueError("spin must be 0, 1 or 2")


def running_width(model, res, x):
    q = daughter_momentum(x, model.m1, model.m2)
    q_r = daughter_momentum(res.mass ** 2, model.m1, model.m2)
    b = blatt_weisskopf(res.spin, q, q_r, res.radius)
    return res.width * (q / q_r) ** (2 * res.spin + 1) * (res.mass / np.sqrt(x)) * b * b


def dynamical(model, res, x):
    """Barrier factors over the Breit-Wigner denominator (everything but the angular factor)."""
    q = daughter_momentum(x, model.m1, model.m2)
    q_r = daughter_momentum(res.mass ** 2, model.m1, model.m2)
    p = bachelor_momentum(x, model.M, model.m3)
    p_r = bachelor_momentum(res.mass ** 2, model.M, model.m3)
    num = blatt_weisskopf(res.spin, q, q_r, res.radius) * blatt_weisskopf(res.spin, p, p_r, model.rD)
    den = res.mass ** 2 - x - 1j * res.mass * running_width(model, res, x)
    return num / den


def breit_wigner(model, res, x, y):
    return dynamical(model, res, x) * zemach(model, res.spin, x, y)


def symmetrised(model, res, s12, s13):
    return breit_wigner(model, res, s12, s13) + breit_wigner(model, res, s13, s12)
