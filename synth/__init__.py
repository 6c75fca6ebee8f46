"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the amplitude method itself: no spline, no
Breit-Wigner, no likelihood.  It defines the decay constants and resonance
tables of the synthetic workloads, draws their seeded parameters, generates
uniform phase-space points (the region test below is the polynomial
cos(theta) <= 1 form, written independently of the oracle's momentum-limit form),
and builds the synthetic detector-efficiency models.  Every random draw uses
``numpy.random.Generator(PCG64(seed))``.

The paper (Sec. 4) studies D+ -> K+K+K-; the throughput workloads follow the
three-body D+ -> pi- pi+ pi+ case with a spline S-wave and P/D-wave
resonances.  Particle 1 is the negatively charged hadron, so both s12 and s13
are m^2(h+ h-) (Sec. 2, definition below Eq. 1; Sec. 4 symmetrisation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

M_DPLUS = 1.86966
M_PI = 0.13957
M_K = 0.493677
R_D = 5.0          # D-meson barrier radius, GeV^-1
R_RES = 1.5        # resonance barrier radius, GeV^-1


@dataclass(frozen=True)
class Resonance:
    name: str
    spin: int
    mass: float
    width: float
    radius: float = R_RES


RHO770 = Resonance("rho(770)", 1, 0.775, 0.149)
F2_1270 = Resonance("f2(1270)", 2, 1.2755, 0.1867)
RHO1450 = Resonance("rho(1450)", 1, 1.465, 0.4)
PHI1020 = Resonance("phi(1020)", 1, 1.019461, 0.004249)
# scalars of an isobar S-wave (Sec. 2 names the form, not the states): synthetic values near the
# f0(980) and f0(1370), plain Breit-Wigners
F0_980 = Resonance("f0(980)", 0, 0.990, 0.060)
F0_1370 = Resonance("f0(1370)", 0, 1.350, 0.350)


@dataclass(frozen=True)
class Decay:
    """Masses in GeV: mother M and daughters m1 (h-), m2 = m3 (the two identical h+)."""
    M: float
    m1: float
    m2: float
    m3: float
    rD: float = R_D

    @property
    def smin(self) -> float:
        return (self.m1 + self.m2) ** 2

    @property
    def smax(self) -> float:
        return (self.M - self.m3) ** 2


D_PIPIPI = Decay(M_DPLUS, M_PI, M_PI, M_PI)
D_KKK = Decay(M_DPLUS, M_K, M_K, M_K)


def uniform_knots(decay: Decay, n_knots: int) -> np.ndarray:
    """N knots evenly spaced from the lower to the upper end of the m^2(h+h-) range."""
    return decay.smin + (decay.smax - decay.smin) * np.arange(n_knots) / (n_knots - 1)


# ---------------------------------------------------------------------------
# phase-space region (polynomial form, no square roots)

def _kallen(a, b, c):
    return a * a + b * b + c * c - 2.0 * (a * b + b * c + c * a)


def inside_region(decay: Decay, s12, s13):
    """True where (s12, s13) is kinematically allowed.

    In the (12) rest frame, s13 - m1^2 - m3^2 = 2(E1 E3 - p1 p3 cos(theta)).  The point is
    physical when |cos(theta)| <= 1, i.e. when
    [2 s12 (s13 - m1^2 - m3^2) - (s12 + m1^2 - m2^2)(M^2 - s12 - m3^2)]^2
        <= lambda(s12, m1^2, m2^2) * lambda(M^2, s12, m3^2).
    """
    s12 = np.asarray(s12, dtype=np.float64)
    s13 = np.asarray(s13, dtype=np.float64)
    M2, a, b, c = decay.M ** 2, decay.m1 ** 2, decay.m2 ** 2, decay.m3 ** 2
    l12 = _kallen(s12, a, b)
    l3 = _kallen(M2, s12, c)
    lhs = 2.0 * s12 * (s13 - a - c) - (s12 + a - b) * (M2 - s12 - c)
    ok = (s12 >= decay.smin) & (s12 <= decay.smax) & (l12 >= 0) & (l3 >= 0)
    return ok & (lhs * lhs <= l12 * l3)


def grid_points(decay: Decay, spacing: float):
    """Evenly spaced normalisation points (Sec. 4): the centres of the square cells of side `spacing`
    (GeV^2) of a grid anchored at (s_min, s_min) that lie inside the Dalitz region, each weighted by
    the cell area spacing^2.  Fig. 2 uses spacings of 0.01, 0.004 and 0.001 GeV^2.

    Returns (s12, s13, w), row by row in s12 and, within a row, increasing s13."""
    lo, hi = decay.smin, decay.smax
    n = int(math.ceil((hi - lo) / spacing))
    c = lo + (np.arange(n) + 0.5) * spacing
    c = c[c <= hi]
    out12, out13 = [], []
    for x in c:
        keep = inside_region(decay, np.full(len(c), x), c)
        if keep.any():
            out13.append(c[keep])
            out12.append(np.full(int(keep.sum()), x))
    s12 = np.concatenate(out12)
    s13 = np.concatenate(out13)
    return s12, s13, np.full(len(s12), spacing * spacing)


def uniform_phase_space(decay: Decay, n: int, seed: int, block: int = 1 << 20):
    """n points uniform in the Dalitz region: box candidates kept if inside, in stream order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = decay.smin, decay.smax
    out12, out13, have = [], [], 0
    while have < n:
        u = rng.uniform(lo, hi, (block, 2))
        keep = inside_region(decay, u[:, 0], u[:, 1])
        u = u[keep]
        out12.append(u[:, 0])
        out13.append(u[:, 1])
        have += len(u)
    return np.concatenate(out12)[:n].copy(), np.concatenate(out13)[:n].copy()


def box_acceptance(decay: Decay, n: int = 1 << 22, seed: int = 7) -> float:
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(decay.smin, decay.smax, (n, 2))
    return float(inside_region(decay, u[:, 0], u[:, 1]).mean())


def region_area_mc(decay: Decay, n: int = 1 << 22, seed: int = 7) -> float:
    return box_acceptance(decay, n, seed) * (decay.smax - decay.smin) ** 2


# ---------------------------------------------------------------------------
# synthetic efficiency models (inputs: the detector response is given, not computed by the method)

@dataclass(frozen=True)
class PolyEfficiency:
    """Symmetric cubic polynomial efficiency in [0.3, 1].

    u = (s12 - smin)/(smax - smin), v likewise; p = sum_{0<=i<=j, i+j<=3} a_ij (u^i v^j + u^j v^i);
    eps = clip(0.3 + 0.7 (p - p_lo)/(p_hi - p_lo), 0.3, 1), with p_lo, p_hi the extremes of p over the
    in-region nodes of a 1001 x 1001 (u, v) grid.
    """
    decay: Decay
    coef: tuple
    p_lo: float
    p_hi: float

    PAIRS = ((0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2))

    @staticmethod
    def _p(coef, u, v):
        p = np.zeros_like(u)
        for a, (i, j) in zip(coef, PolyEfficiency.PAIRS):
            p = p + a * (u ** i * v ** j + u ** j * v ** i)
        return p

    @classmethod
    def seeded(cls, decay: Decay, seed: int) -> "PolyEfficiency":
        rng = np.random.Generator(np.random.PCG64(seed))
        coef = tuple(float(x) for x in rng.uniform(-1.0, 1.0, 6))
        g = np.linspace(0.0, 1.0, 1001)
        uu, vv = np.meshgrid(g, g, indexing="ij")
        span = decay.smax - decay.smin
        inside = inside_region(decay, decay.smin + span * uu, decay.smin + span * vv)
        p = cls._p(coef, uu[inside], vv[inside])
        return cls(decay, coef, float(p.min()), float(p.max()))

    def __call__(self, s12, s13):
        span = self.decay.smax - self.decay.smin
        u = (np.asarray(s12, dtype=np.float64) - self.decay.smin) / span
        v = (np.asarray(s13, dtype=np.float64) - self.decay.smin) / span
        p = self._p(self.coef, u, v)
        return np.clip(0.3 + 0.7 * (p - self.p_lo) / (self.p_hi - self.p_lo), 0.3, 1.0)


def efficiency_histogram(eff: PolyEfficiency, nbins: int = 200) -> np.ndarray:
    """nbins x nbins float32 table of eff at the bin centres over [smin, smax]^2 (index [i12, i13])."""
    d = eff.decay
    delta = (d.smax - d.smin) / nbins
    c = d.smin + (np.arange(nbins) + 0.5) * delta
    cc12, cc13 = np.meshgrid(c, c, indexing="ij")
    return eff(cc12, cc13).astype(np.float32)


# ---------------------------------------------------------------------------
# parameter vectors: [a_0, phi_0, ..., a_{N-1}, phi_{N-1}, |c_1|, arg c_1, ..., m_1, G_1, ...]

def n_params(n_knots: int, n_res: int) -> int:
    return 2 * n_knots + 4 * n_res


# Magnitudes of the resonance coefficients used as "truth".  They are synthetic inputs, picked so
# that, with knot magnitudes drawn from U(0.5, 2), rho(770) carries roughly half the rate of the
# S-wave and the other waves a few to ten per cent of it.  In K-K+K+ the phi(1020) magnitude gives it
# about 10% of the rate and the S-wave about 90%, the split Sec. 4 reports.
TRUTH_C_MAG = {"rho(770)": 0.16, "f2(1270)": 0.32, "rho(1450)": 0.4, "phi(1020)": 0.055,
               "f0(980)": 0.25, "f0(1370)": 0.6}


def truth_theta(n_knots: int, resonances, seed: int) -> np.ndarray:
    """Draw a_k ~ U(0.5, 2), phi_k ~ U(-pi, pi), then arg c of each non-reference resonance ~ U(-pi, pi).

    The first resonance is the phase reference (arg c = 0).  Masses and widths are the table values.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.5, 2.0, n_knots)
    phi = rng.uniform(-math.pi, math.pi, n_knots)
    args = rng.uniform(-math.pi, math.pi, max(len(resonances) - 1, 0))
    th = np.empty(n_params(n_knots, len(resonances)))
    th[0:2 * n_knots:2] = a
    th[1:2 * n_knots:2] = phi
    o = 2 * n_knots
    for r, res in enumerate(resonances):
        th[o + 2 * r] = TRUTH_C_MAG[res.name]
        th[o + 2 * r + 1] = 0.0 if r == 0 else args[r - 1]
    o += 2 * len(resonances)
    for r, res in enumerate(resonances):
        th[o + 2 * r] = res.mass
        th[o + 2 * r + 1] = res.width
    return th


def perturb_theta(theta: np.ndarray, n_knots: int, n_res: int, seed: int) -> np.ndarray:
    """Seeded fit start: a x U(0.8,1.2), phi + U(-0.3,0.3), |c| x U(0.8,1.2), arg c + U(-0.3,0.3),
    m + U(-0.005,0.005), Gamma x U(0.9,1.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    th = np.array(theta, dtype=np.float64, copy=True)
    th[0:2 * n_knots:2] *= rng.uniform(0.8, 1.2, n_knots)
    th[1:2 * n_knots:2] += rng.uniform(-0.3, 0.3, n_knots)
    o = 2 * n_knots
    th[o:o + 2 * n_res:2] *= rng.uniform(0.8, 1.2, n_res)
    th[o + 1:o + 2 * n_res:2] += rng.uniform(-0.3, 0.3, n_res)
    o += 2 * n_res
    th[o:o + 2 * n_res:2] += rng.uniform(-0.005, 0.005, n_res)
    th[o + 1:o + 2 * n_res:2] *= rng.uniform(0.9, 1.1, n_res)
    return th


def fit_start(theta: np.ndarray, n_knots: int, n_res: int, seed: int, float_shapes: bool = False) -> np.ndarray:
    """Seeded start of a toy fit: perturb_theta for the floated parameters, while the held ones (the
    reference coefficient; the masses and widths unless floated) keep the values the toy was generated
    with, as a fit holds them at the model's known values."""
    th = perturb_theta(theta, n_knots, n_res, seed)
    held = fixed_mask(n_knots, n_res, float_shapes).astype(bool)
    th[held] = np.asarray(theta, dtype=np.float64)[held]
    return th


def fixed_mask(n_knots: int, n_res: int, float_shapes: bool = False) -> np.ndarray:
    """1 = held fixed.  The first resonance coefficient is the reference (global phase and scale);
    masses and widths are fixed unless float_shapes."""
    fx = np.zeros(n_params(n_knots, n_res), dtype=np.uint8)
    o = 2 * n_knots
    if n_res:
        fx[o:o + 2] = 1
    if not float_shapes:
        fx[o + 2 * n_res:] = 1
    return fx


# ---------------------------------------------------------------------------
# the workloads

@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    precision: str            # "fp64" or "mixed"
    n_events: int
    n_norm: int
    n_knots: int
    resonances: tuple
    efficiency: str           # "flat", "poly" or "hist"
    float_shapes: bool = False
    decay: Decay = field(default=D_PIPIPI)

    def seed(self, what: str) -> int:
        off = {"truth": 1, "events": 2, "norm": 3, "eff": 4, "start": 5}[what]
        return 100 * self.index + off

    @property
    def n_res(self) -> int:
        return len(self.resonances)

    @property
    def n_params(self) -> int:
        return n_params(self.n_knots, self.n_res)

    def knots(self) -> np.ndarray:
        return uniform_knots(self.decay, self.n_knots)

    def truth(self) -> np.ndarray:
        return truth_theta(self.n_knots, self.resonances, self.seed("truth"))

    def start(self) -> np.ndarray:
        return perturb_theta(self.truth(), self.n_knots, self.n_res, self.seed("start"))

    def fixed(self) -> np.ndarray:
        return fixed_mask(self.n_knots, self.n_res, self.float_shapes)

    def norm_points(self, n: int | None = None):
        return uniform_phase_space(self.decay, self.n_norm if n is None else n, self.seed("norm"))

    def poly_efficiency(self) -> PolyEfficiency:
        return PolyEfficiency.seeded(self.decay, self.seed("eff"))


# Sizes follow the five benchmark configurations of the method: a small fit, a 1M-event FP64 case,
# the 10M-event mixed-precision headline, a 5M-event shape-floating gradient case, and serving.
C1 = Workload("dpipipi_10k_fit", 1, "fp64", 10_000, 100_000, 20, (RHO770, F2_1270), "flat")
C2 = Workload("dpipipi_1M_fp64", 2, "fp64", 1_000_000, 2_000_000, 40, (RHO770, F2_1270, RHO1450), "poly")
C3 = Workload("dpipipi_10M_mixed", 3, "mixed", 10_000_000, 10_000_000, 50, (RHO770, F2_1270), "hist")
C4 = Workload("dpipipi_5M_shapes", 4, "fp64", 5_000_000, 5_000_000, 50, (RHO770, F2_1270, RHO1450), "flat",
              float_shapes=True)
# The decay studied in the paper (Sec. 4): D+ -> K- K+ K+, 40 knots, phi(1020) P-wave, 100k toy events.
KKK = Workload("dkkk_100k", 6, "fp64", 100_000, 1_000_000, 40, (PHI1020,), "flat", decay=D_KKK)
# isobar S-wave (constant non-resonant term + the two scalars) with the P and D waves of C1; the
# two "knots" only carry the constant in the library's isobar form
ISO = Workload("dpipipi_isobar", 7, "fp64", 10_000, 100_000, 2, (F0_980, F0_1370, RHO770, F2_1270), "flat")
WORKLOADS = {w.index: w for w in (C1, C2, C3, C4, KKK, ISO)}


def isobar_truth(resonances, seed: int) -> np.ndarray:
    """Isobar-form parameters [|c_NR|, arg c_NR, (|c_r|, arg c_r)_r, (m_r, Gamma_r)_r]: c_NR = 1 at a
    phase drawn from U(-pi, pi), the first resonance the phase reference, the other phases drawn from
    U(-pi, pi), table masses and widths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = len(resonances)
    th = np.empty(2 + 4 * R)
    th[0], th[1] = 1.0, rng.uniform(-math.pi, math.pi)
    args = rng.uniform(-math.pi, math.pi, max(R - 1, 0))
    for r, res in enumerate(resonances):
        th[2 + 2 * r] = TRUTH_C_MAG[res.name]
        th[3 + 2 * r] = 0.0 if r == 0 else args[r - 1]
    for r, res in enumerate(resonances):
        th[2 + 2 * R + 2 * r] = res.mass
        th[3 + 2 * R + 2 * r] = res.width
    return th


def isobar_fixed(n_res: int, float_shapes: bool = False) -> np.ndarray:
    """1 = held fixed: the first resonance coefficient (phase and scale reference) and, unless
    float_shapes, the masses and widths."""
    fx = np.zeros(2 + 4 * n_res, dtype=np.uint8)
    if n_res:
        fx[2:4] = 1
    if not float_shapes:
        fx[2 + 2 * n_res:] = 1
    return fx

# Serving workload: 256 toy-fit jobs, event counts log-uniform in [1e4, 5e6], knots in {20,30,40,50},
# model as the small fit, shapes fixed, shared normalisation sample.
SERVE_SEED = 501
SERVE_NORM_SEED = 503


def serving_jobs(n_jobs: int = 256, lo: float = 1e4, hi: float = 5e6, seed: int = SERVE_SEED):
    rng = np.random.Generator(np.random.PCG64(seed))
    n_ev = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_jobs))).astype(np.int64)
    knots = rng.choice(np.array([20, 30, 40, 50]), n_jobs)
    return [(int(n), int(k), 10_000 + i) for i, (n, k) in enumerate(zip(n_ev, knots))]


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))
