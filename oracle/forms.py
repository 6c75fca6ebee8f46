"""Alternative S-wave forms (test infrastructure only).

Cartesian knots.  The abstract's source text names, beside the magnitudes and phases of the knot
values, their real and imaginary parts as parameters.  theta_c = [Re z_0, Im z_0, ..., Re z_{N-1},
Im z_{N-1}, |c_1|, arg c_1, ..., m_1, G_1, ...]: the same spline model, other coordinates.  With
G_z = df/dRe z + i df/dIm z (the complex partial of the likelihood module), df/dRe z_k = Re G_z and
df/dIm z_k = Im G_z.

Isobar S-wave (Sec. 2).  The S-wave of the isobar model is a constant non-resonant term plus
Breit-Wigners for the scalar resonances:
    A = c_NR + sum_r c_r R_r(s12, s13),
with R_r the symmetrised Breit-Wigner of the likelihood module (spin 0 for the scalars) and the
constant entering once (reading: not once per h+h- axis).  theta_i = [|c_NR|, arg c_NR, |c_1|, arg c_1,
..., |c_R|, arg c_R, m_1, G_1, ..., m_R, G_R].  Only the model's kinematics and resonances are used
(no knots).  Gradient: B = 1 for c_NR, B = R_r for c_r (the likelihood module's complex notation);
mass and width partials by five-point differences of R_r.
"""
from __future__ import annotations

import numpy as np

from . import likelihood as L
from .resonance import symmetrised


# ---- Cartesian knots -------------------------------------------------------------------------

def polar_from_cartesian(model, theta_c):
    th = np.array(theta_c, dtype=np.float64, copy=True)
    N = model.n_knots
    x, y = th[0:2 * N:2].copy(), th[1:2 * N:2].copy()
    th[0:2 * N:2] = np.hypot(x, y)
    th[1:2 * N:2] = np.arctan2(y, x)
    return th


def cartesian_nll_and_grad(model, theta_c, events, norm, log_eps_sum=0.0, shapes=True):
    th = polar_from_cartesian(model, theta_c)
    s12, s13 = events
    n = len(s12)
    ns12, ns13, w = norm

    def data_seed(a, lo, hi):
        aa = a.real ** 2 + a.imag ** 2
        return -4.0 * a / aa, float(np.sum(np.log(aa)))

    def norm_seed(a, lo, hi):
        return 4.0 * w[lo:hi] * a, float(np.sum(w[lo:hi] * (a.real ** 2 + a.imag ** 2)))

    gz_d, gc_d, gs_d, sum_log = L._accumulate(model, th, s12, s13, data_seed, shapes)
    gz_n, gc_n, gs_n, I = L._accumulate(model, th, ns12, ns13, norm_seed, shapes)
    scale = n / I
    value = -2.0 * sum_log - 2.0 * log_eps_sum + 2.0 * n * np.log(I)
    grad = L._to_params(model, th, gz_d + scale * gz_n, gc_d + scale * gc_n, gs_d + scale * gs_n)
    gz = gz_d + scale * gz_n
    N = model.n_knots
    grad[0:2 * N:2] = gz.real
    grad[1:2 * N:2] = gz.imag
    return value, grad


# ---- Isobar S-wave ---------------------------------------------------------------------------

def _unpack_isobar(model, theta):
    th = np.asarray(theta, dtype=np.float64)
    R = model.n_res
    c_nr = th[0] * np.cos(th[1]) + 1j * (th[0] * np.sin(th[1]))
    cm, ca = th[2:2 + 2 * R:2], th[3:3 + 2 * R:2]
    c = cm * np.cos(ca) + 1j * (cm * np.sin(ca))
    o = 2 + 2 * R
    return c_nr, c, th[o:o + 2 * R:2].copy(), th[o + 1:o + 2 * R:2].copy()


def isobar_components(model, theta, s12, s13):
    c_nr, c, masses, widths = _unpack_isobar(model, theta)
    m = model.with_shapes(masses, widths)
    rs = [symmetrised(m, r, s12, s13) for r in m.res]
    a = np.full(np.shape(s12), c_nr, dtype=np.complex128)
    for cr, rr in zip(c, rs):
        a = a + cr * rr
    return rs, a


def isobar_amplitude(model, theta, s12, s13):
    return isobar_components(model, theta, s12, s13)[1]


def _isobar_shape_derivative(model, theta, r, s12, s13, which):
    _, _, masses, widths = _unpack_isobar(model, theta)
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


def _isobar_accumulate(model, theta, s12, s13, seed_fn, shapes):
    R = model.n_res
    _, c, _, _ = _unpack_isobar(model, theta)
    g_nr = 0.0 + 0.0j
    gc = np.zeros(R, dtype=np.complex128)
    gshape = np.zeros((R, 2))
    extra = 0.0
    for lo, hi in L._chunks(len(s12)):
        x12, x13 = s12[lo:hi], s13[lo:hi]
        rs, a = isobar_components(model, theta, x12, x13)
        g, e = seed_fn(a, lo, hi)
        extra += e
        g_nr += np.sum(g)
        for r in range(R):
            gc[r] += np.sum(g * np.conj(rs[r]))
            if shapes:
                for which in (0, 1):
                    d = _isobar_shape_derivative(model, theta, r, x12, x13, which)
                    gshape[r, which] += float(np.sum((np.conj(g) * c[r] * d).real))
    return g_nr, gc, gshape, extra


def isobar_nll_and_grad(model, theta, events, norm, log_eps_sum=0.0, shapes=True):
    th = np.asarray(theta, dtype=np.float64)
    R = model.n_res
    s12, s13 = events
    n = len(s12)
    ns12, ns13, w = norm

    def data_seed(a, lo, hi):
        aa = a.real ** 2 + a.imag ** 2
        return -4.0 * a / aa, float(np.sum(np.log(aa)))

    def norm_seed(a, lo, hi):
        return 4.0 * w[lo:hi] * a, float(np.sum(w[lo:hi] * (a.real ** 2 + a.imag ** 2)))

    gnr_d, gc_d, gs_d, sum_log = _isobar_accumulate(model, th, s12, s13, data_seed, shapes)
    gnr_n, gc_n, gs_n, I = _isobar_accumulate(model, th, ns12, ns13, norm_seed, shapes)
    scale = n / I
    value = -2.0 * sum_log - 2.0 * log_eps_sum + 2.0 * n * np.log(I)
    out = np.zeros(2 + 4 * R)
    G = gnr_d + scale * gnr_n
    out[0] = G.real * np.cos(th[1]) + G.imag * np.sin(th[1])
    out[1] = th[0] * (-G.real * np.sin(th[1]) + G.imag * np.cos(th[1]))
    gc = gc_d + scale * gc_n
    cm, ca = th[2:2 + 2 * R:2], th[3:3 + 2 * R:2]
    out[2:2 + 2 * R:2] = gc.real * np.cos(ca) + gc.imag * np.sin(ca)
    out[3:3 + 2 * R:2] = cm * (-gc.real * np.sin(ca) + gc.imag * np.cos(ca))
    gs = gs_d + scale * gs_n
    o = 2 + 2 * R
    out[o:o + 2 * R:2] = gs[:, 0]
    out[o + 1:o + 2 * R:2] = gs[:, 1]
    return value, out


def isobar_nll(model, theta, events, norm, log_eps_sum=0.0):
    s12, s13 = events
    a = isobar_amplitude(model, theta, s12, s13)
    ns12, ns13, w = norm
    an = isobar_amplitude(model, theta, ns12, ns13)
    I = float(np.sum(w * (an.real ** 2 + an.imag ** 2)))
    return -2.0 * float(np.sum(np.log(a.real ** 2 + a.imag ** 2))) - 2.0 * log_eps_sum + 2.0 * len(s12) * np.log(I)
