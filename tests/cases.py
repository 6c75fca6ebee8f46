"""Seeded problems shared by the GPU parity tests: the same inputs go to the oracle and to the library."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synth
from oracle import kinematics as K
from oracle import likelihood as L
from tests.conftest import oracle_model


@dataclass
class Problem:
    workload: object
    model: object           # oracle model
    knots: np.ndarray
    theta: np.ndarray
    events: tuple           # (s12, s13)
    eff_events: np.ndarray | None
    norm: tuple             # (s12, s13, w)
    eff_norm: np.ndarray | None
    table: np.ndarray | None = None

    @property
    def log_eps_sum(self):
        return 0.0 if self.eff_events is None else float(np.sum(np.log(self.eff_events)))

    def oracle_norm(self):
        s12, s13, w = self.norm
        return (s12, s13, w if self.eff_norm is None else w * self.eff_norm)

    def oracle(self, theta=None, shapes=False):
        th = self.theta if theta is None else theta
        return L.nll_and_grad(self.model, th, self.events, self.oracle_norm(), self.log_eps_sum, shapes=shapes)

    def nll_scale(self, theta=None):
        """2 sum_i |ln|A_i|^2| + 2 n |ln I|: the size of the terms whose sum is -2 ln L.  Rounding in the
        working precision is relative to this, not to -2 ln L itself, which can cancel to near zero."""
        th = self.theta if theta is None else theta
        a = L.amplitude(self.model, th, *self.events)
        I = L.norm_integral(self.model, th, self.oracle_norm())
        n = len(self.events[0])
        return 2.0 * float(np.sum(np.abs(np.log(a.real ** 2 + a.imag ** 2)))) + 2.0 * n * abs(np.log(I))

    def grad_scale(self, theta=None):
        """Per parameter (knots and coefficients; shapes 0): the sum over points of the magnitudes of
        the terms whose sum is the gradient, |g_p| |dA_p/dtheta| with the data seed |g| = 4/|A| and the
        normalisation seed (n/I) 4 w |A|.  Rounding of FP32 inputs shared by all points (a coefficient,
        cached amplitudes) is coherent across those terms, so the mixed-precision error of a component
        whose data and normalisation sums cancel scales with this, not with the gradient."""
        from oracle import spline as sp
        th = self.theta if theta is None else theta
        m = self.model
        N, R = m.n_knots, m.n_res
        z, c, _, _ = m.unpack(th)
        n = len(self.events[0])
        n12, n13, w = self.oracle_norm()
        I = L.norm_integral(m, th, (n12, n13, w))
        kn = m.knot_array
        out = np.zeros(m.n_params)
        for (s12, s13), seed in ((self.events, lambda a: 4.0 / np.abs(a)),
                                 ((n12, n13), lambda a: (n / I) * 4.0 * w * np.abs(a))):
            _, rs, a = L.components(m, th, s12, s13)
            g = seed(a)
            bz = np.abs(sp.basis_adjoint(kn, s12, g.astype(complex))) + np.abs(sp.basis_adjoint(kn, s13, g.astype(complex)))
            out[0:2 * N:2] += bz
            out[1:2 * N:2] += np.abs(z) * bz
            for r in range(R):
                t = float(np.sum(g * np.abs(rs[r])))
                out[2 * N + 2 * r] += t
                out[2 * N + 2 * r + 1] += abs(c[r]) * t
        return out

    def context(self, precision, table_mode=False):
        from paper_1703_03284_amd import context_for
        ctx = context_for(self.workload.decay, self.knots, self.workload.resonances, precision)
        if table_mode:
            d = self.workload.decay
            ctx.set_eff_table(self.table, d.smin, d.smax)
            ctx.load_events(*self.events)
            ctx.load_norm(*self.norm)
        else:
            ctx.load_events(*self.events, eff=self.eff_events)
            ctx.load_norm(*self.norm, eff=self.eff_norm)
        ctx.set_params(self.theta)
        return ctx


def make_problem(workload, n_events, n_norm, seed=0, knots=None, eff="auto", theta=None):
    kn = workload.knots() if knots is None else np.asarray(knots, dtype=np.float64)
    m = oracle_model(workload, knots=kn)
    ev = synth.uniform_phase_space(workload.decay, n_events, 1000 + seed)
    s12, s13 = synth.uniform_phase_space(workload.decay, n_norm, 2000 + seed)
    w = np.full(n_norm, K.area(m) / n_norm)
    mode = workload.efficiency if eff == "auto" else eff
    e_ev = e_nm = table = None
    if mode in ("poly", "hist"):
        pe = synth.PolyEfficiency.seeded(workload.decay, workload.seed("eff"))
        if mode == "poly":
            e_ev, e_nm = pe(*ev), pe(s12, s13)
        else:
            table = synth.efficiency_histogram(pe)
            d = workload.decay
            e_ev = L.hist_lookup(table, d.smin, d.smax, *ev)
            e_nm = L.hist_lookup(table, d.smin, d.smax, s12, s13)
    th = workload.start() if theta is None else theta
    if len(th) != 2 * len(kn) + 4 * workload.n_res:
        th = synth.perturb_theta(synth.truth_theta(len(kn), workload.resonances, workload.seed("truth")),
                                 len(kn), workload.n_res, workload.seed("start"))
    return Problem(workload, m, kn, th, ev, e_ev, (s12, s13, w), e_nm, table)


def with_grid_norm(prob: Problem, spacing: float) -> Problem:
    """The same problem normalised on the evenly spaced grid of the given spacing (Sec. 4), flat
    efficiency."""
    g = synth.grid_points(prob.workload.decay, spacing)
    return Problem(prob.workload, prob.model, prob.knots, prob.theta, prob.events, None, g, None, None)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)
