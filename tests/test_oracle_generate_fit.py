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
