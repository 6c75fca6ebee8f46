"""Model description used by the oracle (test infrastructure only).

A model is the decay kinematics (mother M, daughters m1 = h-, m2 = m3 = the identical h+), the
D-meson barrier radius, the S-wave knot positions (Sec. 2: N boundary points covering the
m^2(h+h-) spectrum) and the list of P/D-wave resonances (Sec. 2: spin-dependent Breit-Wigners).

Parameter vector layout (2N + 4R reals):
  [a_0, phi_0, ..., a_{N-1}, phi_{N-1},  |c_1|, arg c_1, ..., |c_R|, arg c_R,  m_1, G_1, ..., m_R, G_R]
The knot pairs are the paper's {a_k, phi_k} (Sec. 2); the resonance coefficients c_k^L of Eq. 1 are
taken in polar form to match the knots.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Res:
    spin: int
    mass: float
    width: float
    radius: float


@dataclass(frozen=True)
class Model:
    M: float
    m1: float
    m2: float
    m3: float
    rD: float
    knots: tuple
    res: tuple

    @property
    def n_knots(self) -> int:
        return len(self.knots)

    @property
    def n_res(self) -> int:
        return len(self.res)

    @property
    def n_params(self) -> int:
        return 2 * self.n_knots + 4 * self.n_res

    @property
    def knot_array(self) -> np.ndarray:
        return np.asarray(self.knots, dtype=np.float64)

    def unpack(self, theta):
        """theta -> (z_k complex knot values, c_r complex coefficients, masses, widths)."""
        th = np.asarray(theta, dtype=np.float64)
        N, R = self.n_knots, self.n_res
        a, phi = th[0:2 * N:2], th[1:2 * N:2]
        z = a * np.cos(phi) + 1j * (a * np.sin(phi))
        o = 2 * N
        cm, ca = th[o:o + 2 * R:2], th[o + 1:o + 2 * R:2]
        c = cm * np.cos(ca) + 1j * (cm * np.sin(ca))
        o += 2 * R
        return z, c, th[o:o + 2 * R:2].copy(), th[o + 1:o + 2 * R:2].copy()

    def with_shapes(self, masses, widths) -> "Model":
        return Model(self.M, self.m1, self.m2, self.m3, self.rD, self.knots,
                     tuple(Res(r.spin, float(m), float(g), r.radius)
                           for r, m, g in zip(self.res, masses, widths)))
