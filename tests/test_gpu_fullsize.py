"""Checks at the benchmark workloads' full sizes, in the launch configuration bench.py times.

The oracle computes -2 ln L and the knot and coefficient gradient at 10M + 10M points and at 1M + 2M
points, and at 5M + 5M with masses and widths floated the whole gradient including the mass and width
partials (its per-point five-point differences split over the host's cores by oracle.pool); there the
FP64 adjoint is also checked against central differences of the library's FP64 -2 ln L, and the
mixed-precision gradient against the FP64 one.
"""
import numpy as np
import pytest

import synth
from oracle import kinematics as K
from oracle import likelihood as L
from tests.cases import make_problem, rel
from tests.conftest import oracle_model

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _prec(name):
    from paper_1703_03284_amd import FP64, MIXED
    return {"fp64": FP64, "mixed": MIXED}[name]


@pytest.fixture(scope="module")
def headline():
    wl = synth.C3
    d = wl.decay
    m = oracle_model(wl)
    table = synth.efficiency_histogram(synth.PolyEfficiency.seeded(d, wl.seed("eff")))
    ev = synth.uniform_phase_space(d, wl.n_events, 31)
    s12, s13 = synth.uniform_phase_space(d, wl.n_norm, wl.seed("norm"))
    w = np.full(len(s12), K.area(m) / len(s12))
    e_ev = L.hist_lookup(table, d.smin, d.smax, *ev)
    e_nm = L.hist_lookup(table, d.smin, d.smax, s12, s13)
    th = wl.start()
    v_o, g_o = L.nll_and_grad(m, th, ev, (s12, s13, w * e_nm), float(np.sum(np.log(e_ev))), shapes=False)
    return wl, table, ev, (s12, s13, w), th, v_o, g_o


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-6), ("fp64", 1e-10)])
def test_headline_nll_full_size(headline, prec, tol):
    from paper_1703_03284_amd import context_for
    wl, table, ev, nm, th, v_o, g_o = headline
    d = wl.decay
    ctx = context_for(d, wl.knots(), wl.resonances, _prec(prec))
    ctx.set_eff_table(table, d.smin, d.smax)
    ctx.load_events(*ev)
    ctx.load_norm(*nm)
    v, g = ctx.eval(th)
    assert rel(v, v_o) <= tol, (v, v_o)
    # the gradient of the knots and coefficients against the oracle's (shapes fixed: their partials are 0)
    n_ck = 2 * wl.n_knots + 2 * wl.n_res
    g_tol = 1e-8 if prec == "fp64" else 1e-4
    assert np.abs(g[:n_ck] - g_o[:n_ck]).max() <= g_tol * np.abs(g_o[:n_ck]).max()
    assert np.all(g[n_ck:] == 0.0)
    ctx.close()


def test_headline_two_part_sweep_is_bitwise_in_either_order(headline):
    """At 10M + 10M points the sweep reads 520 MB, between one and three times the Infinity Cache, so
    each wave sweeps its tiles in two parts and consecutive evaluations take the parts in opposite
    orders: every other evaluation must give bitwise the same -2 ln L and gradient.  The same sample
    with the quadratic form reads 240 MB, which fits the cache, and is swept in one part."""
    from paper_1703_03284_amd import MIXED, NORM_QFORM, context_for
    wl, table, ev, nm, th, v_o, g_o = headline
    d = wl.decay
    for qform in (False, True):
        ctx = context_for(d, wl.knots(), wl.resonances, MIXED)
        if qform:
            ctx.set_norm_mode(NORM_QFORM)
        ctx.set_eff_table(table, d.smin, d.smax)
        ctx.load_events(*ev)
        ctx.load_norm(*nm)
        runs = [ctx.eval(th) for _ in range(3)]
        for v, g in runs[1:]:
            assert v == runs[0][0] and np.array_equal(g, runs[0][1])
        ctx.close()


def test_headline_mixed_gradient_vs_fp64_full_size(headline):
    from paper_1703_03284_amd import context_for
    wl, table, ev, nm, th, _, _ = headline
    d = wl.decay
    out = {}
    for prec in ("fp64", "mixed"):
        ctx = context_for(d, wl.knots(), wl.resonances, _prec(prec))
        ctx.set_eff_table(table, d.smin, d.smax)
        ctx.load_events(*ev)
        ctx.load_norm(*nm)
        out[prec] = ctx.eval(th)
        ctx.close()
    g64, g32 = out["fp64"][1], out["mixed"][1]
    assert np.abs(g32 - g64).max() <= 1e-4 * np.abs(g64).max()


def test_fp64_gradient_full_size_1m():
    wl = synth.C2
    prob = make_problem(wl, wl.n_events, wl.n_norm, seed=2)
    ctx = prob.context(_prec("fp64"))
    v, g = ctx.eval()
    v_o, g_o = prob.oracle()
    assert rel(v, v_o) <= 1e-10
    n_ck = 2 * wl.n_knots + 2 * wl.n_res
    assert np.abs(g[:n_ck] - g_o[:n_ck]).max() <= 1e-8 * np.abs(g_o[:n_ck]).max()


def test_shape_gradient_full_size_5m():
    from oracle.pool import OraclePool
    from paper_1703_03284_amd import context_for
    wl = synth.C4
    d = wl.decay
    m = oracle_model(wl)
    ev = synth.uniform_phase_space(d, wl.n_events, 41)
    s12, s13 = synth.uniform_phase_space(d, wl.n_norm, wl.seed("norm"))
    w = np.full(len(s12), K.area(m) / len(s12))
    th = wl.start()
    with OraclePool(m, ev, (s12, s13, w)) as pool:
        v_o, g_o = pool.nll_and_grad(th, shapes=True)
    ctxs = {}
    for prec in ("fp64", "mixed"):
        c = context_for(d, wl.knots(), wl.resonances, _prec(prec))
        c.load_events(*ev)
        c.load_norm(s12, s13, w)
        c.set_fixed(wl.fixed())
        ctxs[prec] = c
    v64, g64 = ctxs["fp64"].eval(th)
    v32, g32 = ctxs["mixed"].eval(th)
    # against the oracle: every parameter, the mass and width partials included (the oracle's come from
    # five-point differences of the amplitudes, so the FP64 bound is that of the parity tests with
    # shapes floated)
    assert rel(v64, v_o) <= 1e-10, (v64, v_o)
    assert rel(v32, v_o) <= 1e-6, (v32, v_o)
    assert np.abs(g64 - g_o).max() <= 1e-7 * np.abs(g_o).max(), np.abs(g64 - g_o).max() / np.abs(g_o).max()
    assert np.abs(g32 - g_o).max() <= 1e-4 * np.abs(g_o).max(), np.abs(g32 - g_o).max() / np.abs(g_o).max()
    assert rel(v32, v64) <= 1e-6
    assert np.abs(g32 - g64).max() <= 1e-4 * np.abs(g64).max()
    N, R = wl.n_knots, wl.n_res
    for p in range(2 * N + 2 * R, 2 * N + 4 * R):
        tp, tm = th.copy(), th.copy()
        tp[p] += 1e-6
        tm[p] -= 1e-6
        fd = (ctxs["fp64"].eval(tp)[0] - ctxs["fp64"].eval(tm)[0]) / 2e-6
        assert abs(fd - g64[p]) <= 1e-4 * abs(g64[p]) + 1e-6 * np.abs(g64).max(), (p, fd, g64[p])
    for c in ctxs.values():
        c.close()


def test_torch_autograd_and_device_output():
    import torch
    from paper_1703_03284_amd.torch_nll import MipwaNLL, nll_on_device
    prob = make_problem(synth.C1, 3000, 20000, seed=6)
    ctx = prob.context(_prec("fp64"))
    v, g = ctx.eval(prob.theta)
    theta = torch.tensor(prob.theta, dtype=torch.float64, requires_grad=True)
    out = MipwaNLL.apply(theta, ctx)
    (2.5 * out).backward()
    assert out.item() == v
    np.testing.assert_array_equal(theta.grad.numpy(), 2.5 * g)
    dev = nll_on_device(torch.tensor(prob.theta, dtype=torch.float64), ctx)
    torch.cuda.synchronize()
    host = dev.cpu().numpy()
    assert host[0] == v
    np.testing.assert_array_equal(host[1:], g)


def test_async_evaluation_on_another_stream_is_ordered():
    """An evaluation queued on torch's stream, followed at once (no host synchronisation) by
    synchronous evaluations on the context's own stream at other parameters -- one of them with new
    resonance shapes, which rebuilds the amplitude cache -- gives every result bitwise equal to the
    same evaluations run one after another."""
    import torch
    from paper_1703_03284_amd.torch_nll import nll_on_device
    prob = make_problem(synth.C2, 400_000, 1_000_000, seed=13)
    ctx = prob.context(_prec("mixed"))
    th1 = prob.theta.copy()
    th2 = th1.copy()
    th2[0] *= 1.01
    th3 = th1.copy()
    th3[-3] += 0.004  # a mass: the cache is rebuilt
    seq = [ctx.eval(t) for t in (th1, th2, th3, th1)]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        dev = [nll_on_device(torch.tensor(th1), ctx) for _ in range(3)]
    r2 = ctx.eval(th2)
    with torch.cuda.stream(side):
        dev.append(nll_on_device(torch.tensor(th1), ctx))
    r3 = ctx.eval(th3)
    r1 = ctx.eval(th1)
    torch.cuda.synchronize()
    for d in dev:
        h = d.cpu().numpy()
        assert h[0] == seq[0][0] and np.array_equal(h[1:], seq[0][1])
    for (v, g), (vs, gs) in ((r2, seq[1]), (r3, seq[2]), (r1, seq[3])):
        assert v == vs and np.array_equal(g, gs)
    ctx.close()
