"""Amplitude, -2 ln L, its gradient, component integrals and fit fractions (test infrastructure only).

Sec. 2, Eq. 1: A(s12, s13) = sum_L sum_k c_k^L A_k^L(s12, s13).  Here the S-wave (component 0,
coefficient fixed to 1) is the spline of Sec. 2 evaluated on both h+h- axes and the P/D waves are
the symmetrised Breit-Wigners (Sec. 4):
    A = S(s12) + S(s13) + sum_r c_r R_r(s12, s13).
Sec. 2 and Sec. 4: unbinned maximum likelihood with the PDF normalised to one every iteration.
With detector efficiency eps and normalisation points (s12_j, s13_j) of weight w_j,
    P(x) = |A(x)|^2 eps(x) / I,    I = sum_j w_j eps_j |A(x_j)|^2,
    -2 ln L = -2 sum_i ln|A(x_i)|^2 - 2 sum_i ln eps(x_i) + 2 n ln I.
For uniform phase-space points w_j = |D| / n_norm; for a grid (Sec. 4) w_j is the cell area.

Gradient (complex notation G_v = df/dRe v + i df/dIm v for a complex parameter v entering A
linearly as A = ... + B v):  G_v = sum_p g_p conj(B_p) with the per-point seed
    g = -4 A / |A|^2 on data points,   g = (4 n / I) w eps A on normalisation points.
For a knot value z_k the coefficient B is the (real) cardinal spline basis summed over both axes;
for c_r it is R_r.  The mass and width partials are sum_p Re(conj(g_p) c_r dR_r/dtheta), with
dR_r/dtheta taken from a five-point difference of R_r per point (a deliberately different route from
an analytic derivative).
"""
from __future__ import annotations

import numpy as np

from . import spline as sp
from .resonance import symmetrised

CHUNK = 1 << 20


def components(model, theta, s12, s13):
    """(A_0, [R_r], A) at the points: the S-wave on both axes, the resonance terms and the total."""
    z, c, masses, widths = model.unpack(theta)
    m = model.with_shapes(masses, widths)
    Mpp = sp.second_derivatives(model.knot_array, z)
    a0 = sp.evaluate(model.knot_array, z, Mpp, s12) + sp.evaluate(model.knot_array, z, Mpp, s13)
    rs = [symmetrised(m, r, s12, s13) for r in m.res]
    a = a0.copy()
    for cr, rr in zip(c, rs):
        a = a + cr * rr
    return a0, rs, a


def amplitude(model, theta, s12, s13):
    return components(model, theta, s12, s13)[2]


def _chunks(n):
    for lo in range(0, n, CHUNK):
        yield lo, min(n, lo + CHUNK)


def norm_integral(model, theta, norm):
    s12, s13, w = norm
    tot = 0.0
    for lo, hi in _chunks(len(s12)):
        a = amplitude(model, theta, s12[lo:hi], s13[lo:hi])
        tot += float(np.sum(w[lo:hi] * (a.real ** 2 + a.imag ** 2)))
    return tot


def nll(model, theta, events, norm, log_eps_sum=0.0):
    """-2 ln L.  events = (s12, s13); norm = (s12, s13, w*eps); log_eps_sum = sum_i ln eps(x_i)."""
    s12, s13 = events
    n = len(s12)
    sum_log = 0.0
    for lo, hi in _chunks(n):
        a = amplitude(model, theta, s12[lo:hi], s13[lo:hi])
        sum_log += float(np.sum(np.log(a.real ** 2 + a.imag ** 2)))
    I = norm_integral(model, theta, norm)
    return -2.0 * sum_log - 2.0 * log_eps_sum + 2.0 * n * np.log(I)


def _shape_derivatives(model, theta, r, s12, s13, which):
    """Five-point difference of R_r with respect to its mass (which=0) or width (which=1)."""
    z, c, masses, widths = model.unpack(theta)
    step = 1e-3 * widths[r]
    vals = []
    for k in (-2, -1, 1, 2):
        mm, ww = masses.copy(), widths.copy()
        if which == 0:
            mm[r] += k * step
        else:
            ww[r] += k * step
        m = model.with_shapes(mm, ww)
        vals.append(symmetrised(m, m.res[r], s12, s13))
    return (vals[0] - 8.0 * vals[1] + 8.0 * vals[2] - vals[3]) / (12.0 * step)


def _accumulate(model, theta, s12, s13, seed_fn, shapes):
    """Sum over points of the complex partials for one point set, given the per-point seed."""
    N, R = model.n_knots, model.n_res
    z, c, _, _ = model.unpack(theta)
    gz = np.zeros(N, dtype=np.complex128)
    gc = np.zeros(R, dtype=np.complex128)
    gshape = np.zeros((R, 2))
    extra = 0.0
    for lo, hi in _chunks(len(s12)):
        x12, x13 = s12[lo:hi], s13[lo:hi]
        a0, rs, a = components(model, theta, x12, x13)
        g, e = seed_fn(a, lo, hi)
        extra += e
        gz += sp.basis_adjoint(model.knot_array, x12, g) + sp.basis_adjoint(model.knot_array, x13, g)
        for r in range(R):
            gc[r] += np.sum(g * np.conj(rs[r]))
            if shapes:
                for which in (0, 1):
                    d = _shape_derivatives(model, theta, r, x12, x13, which)
                    gshape[r, which] += float(np.sum((np.conj(g) * c[r] * d).real))
    return gz, gc, gshape, extra


def _to_params(model, theta, gz, gc, gshape):
    N, R = model.n_knots, model.n_res
    th = np.asarray(theta, dtype=np.float64)
    out = np.zeros(model.n_params)
    a, phi = th[0:2 * N:2], th[1:2 * N:2]
    out[0:2 * N:2] = gz.real * np.cos(phi) + gz.imag * np.sin(phi)
    out[1:2 * N:2] = a * (-gz.real * np.sin(phi) + gz.imag * np.cos(phi))
    o = 2 * N
    cm, ca = th[o:o + 2 * R:2], th[o + 1:o + 2 * R:2]
    out[o:o + 2 * R:2] = gc.real * np.cos(ca) + gc.imag * np.sin(ca)
    out[o + 1:o + 2 * R:2] = cm * (-gc.real * np.sin(ca) + gc.imag * np.cos(ca))
    o += 2 * R
    out[o:o + 2 * R:2] = gshape[:, 0]
    out[o + 1:o + 2 * R:2] = gshape[:, 1]
    return out


def point_sums(model, theta, s12, s13, w=None, shapes=True):
    """The sums over one set of points that -2 ln L and its gradient are made of: for data points
    (w None) sum ln|A|^2 and the complex partials with the seed -4A/|A|^2; for normalisation points
    of weight w (x efficiency) sum w|A|^2 and the partials with the seed 4 w A, before the n / I scale.
    Returns (gz, gc, gshape, sum).  Sums over disjoint subsets of the points add up to the sums over
    their union."""
    if w is None:
        def seed(a, lo, hi):
            aa = a.real ** 2 + a.imag ** 2
            return -4.0 * a / aa, float(np.sum(np.log(aa)))
    else:
        def seed(a, lo, hi):
            return 4.0 * w[lo:hi] * a, float(np.sum(w[lo:hi] * (a.real ** 2 + a.imag ** 2)))
    return _accumulate(model, theta, s12, s13, seed, shapes)


def combine(model, theta, n_events, data_sums, norm_sums, log_eps_sum=0.0):
    """(-2 ln L, gradient) from the data and normalisation point sums of point_sums:
    -2 ln L = -2 sum ln|A|^2 - 2 sum ln eps + 2 n ln I, gradient = data partials + (n / I) norm partials."""
    gz_d, gc_d, gs_d, sum_log = data_sums
    gz_n, gc_n, gs_n, I = norm_sums
    scale = n_events / I
    value = -2.0 * sum_log - 2.0 * log_eps_sum + 2.0 * n_events * np.log(I)
    grad = _to_params(model, theta, gz_d + scale * gz_n, gc_d + scale * gc_n, gs_d + scale * gs_n)
    return value, grad


def nll_and_grad(model, theta, events, norm, log_eps_sum=0.0, shapes=True):
    """(-2 ln L, gradient over all 2N + 4R parameters).  With shapes=False the mass and width
    partials are left at zero (they are the expensive part of this reference)."""
    s12, s13 = events
    ns12, ns13, w = norm
    return combine(model, theta, len(s12), point_sums(model, theta, s12, s13, None, shapes),
                   point_sums(model, theta, ns12, ns13, w, shapes), log_eps_sum)


def integrals(model, theta, norm):
    """I_jk = sum_p w_p A_j A_k^* over the K = R + 1 components (component 0 = S-wave)."""
    s12, s13, w = norm
    K = model.n_res + 1
    out = np.zeros((K, K), dtype=np.complex128)
    for lo, hi in _chunks(len(s12)):
        a0, rs, _ = components(model, theta, s12[lo:hi], s13[lo:hi])
        comps = [a0] + rs
        for j in range(K):
            for k in range(K):
                out[j, k] += np.sum(w[lo:hi] * comps[j] * np.conj(comps[k]))
    return out


def coefficient_vector(model, theta):
    _, c, _, _ = model.unpack(theta)
    return np.concatenate([[1.0 + 0.0j], c])


def fit_fractions(model, theta, Ibar):
    """FF_jk = Re(c_j c_k^* Ibar_jk) / sum_jk c_j c_k^* Ibar_jk, with c_0 = 1 for the S-wave."""
    c = coefficient_vector(model, theta)
    terms = (np.outer(c, np.conj(c)) * Ibar).real
    return terms / terms.sum()


def hist_lookup(table, lo, hi, s12, s13):
    """Bilinear interpolation between bin centres of an nx x ny table over [lo, hi]^2, constant
    beyond the outermost centres.  Index decisions are taken in FP64."""
    tab = np.asarray(table, dtype=np.float64)
    nx, ny = tab.shape

    def axis(s, nb):
        d = (hi - lo) / nb
        u = (np.asarray(s, dtype=np.float64) - lo) / d - 0.5
        i = np.clip(np.floor(u), 0, nb - 2).astype(np.int64)
        t = np.clip(u - i, 0.0, 1.0)
        return i, t

    i, tx = axis(s12, nx)
    j, ty = axis(s13, ny)
    return ((1 - tx) * (1 - ty) * tab[i, j] + tx * (1 - ty) * tab[i + 1, j]
            + (1 - tx) * ty * tab[i, j + 1] + tx * ty * tab[i + 1, j + 1])
