"""Pins for the oracle's toy generator (Sec. 4 toy MC), its Philox stream, and the fit (Sec. 2, Sec. 4)."""
import json
import os

import numpy as np
import pytest
from scipy.stats import chi2

import synth
from oracle import fit as F
from oracle import generate as G
from oracle import kinematics as K
from oracle import likelihood as L
from oracle.philox import candidate_uniforms, philox4x32_10, to_unit
from tests.conftest import oracle_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    for v in json.load(open(os.path.join(GOLDEN, "philox_kat.json")))["vectors"]:
        c = [np.array([int(x, 16)], dtype=np.uint64) for x in v["ctr"]]
        k = [int(x, 16) for x in v["key"]]
        out = philox4x32_10(*c, *k)
        assert [int(o[0]) for o in out] == [int(x, 16) for x in v["out"]]


def test_unit_mapping():
    assert to_unit(np.array([0]), np.array([0]))[0] == 0.0
    top = to_unit(np.array([0xFFFFFFFF]), np.array([0xFFFFFFFF]))[0]
    assert top == 1.0 - 2.0 ** -53
    u12, u13, v = candidate_uniforms(1234, 0, 200000)
    for u in (u12, u13, v):
        assert 0.0 <= u.min() and u.max() < 1.0
        assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    assert abs(np.corrcoef(u12, u13)[0, 1]) < 0.02


def test_generated_sample_follows_the_density():
    """Chi-square of a 2D histogram of accepted events against |A|^2 integrated per bin by uniform MC."""
    w = synth.C1
    m = oracle_model(w)
    th = w.truth()
    s12, s13, fmax = G.toy(m, th, 20000, seed=42, n_probe=200_000)
    assert len(s12) == 20000 and K.inside(m, s12, s13).all()
    edges = np.linspace(K.smin(m), K.smax(m), 9)
    obs, _, _ = np.histogram2d(s12, s13, bins=[edges, edges])
    u12, u13 = synth.uniform_phase_space(w.decay, 2_000_000, 99)
    a = L.amplitude(m, th, u12, u13)
    exp_w, _, _ = np.histogram2d(u12, u13, bins=[edges, edges], weights=a.real ** 2 + a.imag ** 2)
    exp = exp_w / exp_w.sum() * len(s12)
    keep = exp > 20
    stat = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert chi2.sf(stat, keep.sum() - 1) > 1e-3


def test_accept_reject_draw_for_draw():
    """Accepted candidates are exactly those inside with f > v fmax, in candidate order."""
    w = synth.C1
    m = oracle_model(w)
    th = w.truth()
    fmax = 40.0
    s12, s13, _ = G.accept_reject(m, th, 500, seed=7, fmax=fmax)
    c12, c13, v = G.candidates(m, 7, 0, 1 << 20)
    ok = K.inside(m, c12, c13)
    a = L.amplitude(m, th, c12, c13)
    acc = np.flatnonzero(ok & ((a.real ** 2 + a.imag ** 2) > v * fmax))[:500]
    assert np.array_equal(s12, c12[acc]) and np.array_equal(s13, c13[acc])


@pytest.mark.slow
def test_fit_closure_small_toy():
    """Sec. 4: fitted {a_k, phi_k} compared with the generated inputs (closure within 5 sigma)."""
    w = synth.C1
    m = oracle_model(w)
    truth = w.truth()
    s12, s13, _ = G.toy(m, truth, 5000, seed=w.seed("events"), n_probe=200_000)
    n12, n13 = synth.uniform_phase_space(w.decay, 40000, w.seed("norm"))
    norm = (n12, n13, np.full(len(n12), K.area(m) / len(n12)))
    res = F.fit(m, w.start(), (s12, s13), norm, w.fixed(), gtol=1e-4)
    assert res["edm"] < 1e-3
    free = np.flatnonzero(w.fixed() == 0)
    tc = F.canonical(m, truth)
    d = res["theta"] - tc
    d[1::2][: m.n_knots + m.n_res] = np.angle(np.exp(1j * d[1::2][: m.n_knots + m.n_res]))
    pulls = d[free] / res["sigma"][free]
    assert np.all(np.abs(pulls) < 5), pulls
    assert abs(pulls.mean()) < 1.0


def test_fmax_doubling_restart():
    """With a probe of only three candidates, 1.5 x the probe maximum is below the largest density
    the generator meets, so f_max is doubled and generation restarts from the first candidate.  The
    sample returned is exactly the accept-reject sample at the final f_max (nothing accepted under a
    smaller f_max survives), the final f_max is the probe value times a power of two, and half of it
    would have been exceeded (the last doubling was needed)."""
    w = synth.C1
    m = oracle_model(w)
    th = w.truth()
    probe = G.density_max(m, th, 77 + 1000, 3)
    s12, s13, fmax = G.toy(m, th, 300, seed=77, n_probe=3)
    k = np.log2(fmax / (1.5 * probe))
    assert k >= 1 and k == round(k)
    r12, r13, exceeded = G.accept_reject(m, th, 300, 77, fmax)
    assert not exceeded
    assert np.array_equal(s12, r12) and np.array_equal(s13, r13)
    _, _, exceeded_half = G.accept_reject(m, th, 300, 77, fmax / 2)
    assert exceeded_half
    # every density met on the way to the 300th acceptance is below the final f_max
    c12, c13, _ = G.candidates(m, 77, 0, 1 << 20)
    ok = K.inside(m, c12, c13)
    assert G.density(m, th, c12[ok], c13[ok]).max() <= fmax


@pytest.mark.slow
def test_covariance_matches_inverse_expected_information():
    """The fit's covariance V = 2 H^-1 (H the Hessian of -2 ln L) equals, up to the statistical
    spread of the observed Hessian, the inverse of the expected information n Cov_P(grad ln|A|^2)
    (Sec. 4 judges fitted values by their errors).  The information is computed by brute force, per
    point, from central differences of ln|A|^2 over a large uniform sample weighted by the density:
    no part of it uses the fit's Hessian.  A covariance of H^-1 (a factor 2 off in variance) or one
    taken from the Hessian of -ln L without the factor would fail by a factor of 2."""
    from oracle import Model, Res
    d = synth.D_PIPIPI
    N = 6
    knots = tuple(synth.uniform_knots(d, N))
    m = Model(d.M, d.m1, d.m2, d.m3, d.rD, knots, (Res(1, 0.775, 0.149, 1.5),))
    truth = synth.truth_theta(N, (synth.RHO770,), 4242)
    fixed = synth.fixed_mask(N, 1)
    s12, s13, _ = G.toy(m, truth, 20000, seed=4243, n_probe=200_000)
    n12, n13 = synth.uniform_phase_space(d, 60000, 4244)
    w = np.full(len(n12), K.area(m) / len(n12))
    start = synth.perturb_theta(truth, N, 1, 4245)
    res = F.fit(m, start, (s12, s13), (n12, n13, w), fixed, gtol=1e-6)
    free = np.flatnonzero(fixed == 0)
    th = res["theta_raw"]
    # expected information per event: Cov_P of grad ln|A|^2 over the uniform sample, P = w|A|^2 / I
    u12, u13 = synth.uniform_phase_space(d, 400000, 4246)
    a = L.amplitude(m, th, u12, u13)
    p = a.real ** 2 + a.imag ** 2
    p = p / p.sum()
    grads = np.empty((len(free), len(u12)))
    for i, k in enumerate(free):
        h = 1e-5 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        ap, am = L.amplitude(m, tp, u12, u13), L.amplitude(m, tm, u12, u13)
        grads[i] = (np.log(ap.real ** 2 + ap.imag ** 2) - np.log(am.real ** 2 + am.imag ** 2)) / (2 * h)
    mean = grads @ p
    c = grads - mean[:, None]
    info = len(s12) * (c * p) @ c.T
    v_expected = np.linalg.inv(info)
    v_fit = res["cov"][np.ix_(free, free)]
    ratio = np.diag(v_fit) / np.diag(v_expected)
    assert np.all((ratio > 0.8) & (ratio < 1.25)), ratio
    assert abs(np.median(ratio) - 1.0) < 0.1, ratio
