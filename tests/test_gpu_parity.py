"""GPU library vs the FP64 oracle, element by element on the same seeded inputs.

Tolerances: FP64 mode |d(-2 ln L)| <= 1e-10 relative and ||d grad||_inf <= 1e-8 ||grad||_inf;
mixed mode 1e-6 relative and 1e-4 ||grad||_inf.  The one exception is a likelihood whose terms cancel
(D+ -> K-K+K+ with the narrow phi(1020)): there the mixed bounds are relative to the size of the summed
terms (tests.cases.Problem.nll_scale, grad_scale).  Inputs span many tiles, cells with full tiles and
ragged tails, and points on knots.
"""
import numpy as np
import pytest

import synth
from oracle import generate as OG
from oracle import kinematics as K
from oracle import likelihood as L
from tests.cases import make_problem, rel

pytestmark = pytest.mark.gpu

FP64_NLL, FP64_G = 1e-10, 1e-8
MIX_NLL, MIX_G = 1e-6, 1e-4


def _prec(name):
    from paper_1703_03284_amd import FP64, MIXED
    return {"fp64": FP64, "mixed": MIXED}[name]


def _check(prob, ctx, tol_nll, tol_g, shapes=False, cancelling=False):
    """cancelling: the likelihood's terms cancel (K-K+K+ with phi(1020): -2 ln L of -324 from terms of
    ~2e4), so FP32 rounding, which is relative to the terms, is bounded against their size."""
    v_o, g_o = prob.oracle(shapes=shapes)
    v, g = ctx.eval()
    if cancelling:
        scale = prob.nll_scale()
        assert abs(v - v_o) <= tol_nll * scale, (v, v_o, abs(v - v_o) / scale)
    else:
        assert rel(v, v_o) <= tol_nll, (v, v_o, rel(v, v_o))
    P = len(g_o)
    n_ck = 2 * prob.model.n_knots + 2 * prob.model.n_res
    sel = np.arange(P) if shapes else np.arange(n_ck)
    err = np.abs(g[sel] - g_o[sel])
    bound = tol_g * np.abs(g_o[sel]).max()
    if cancelling:
        bound = bound + 1e-5 * prob.grad_scale()[sel]
    assert np.all(err <= bound), (int(np.argmax(err - bound)), err.max(), np.abs(g_o[sel]).max())
    if not shapes:
        assert np.all(g[n_ck:] == 0.0)
    return v, g


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("wl,n_ev,n_nm", [(synth.C1, 3000, 20000), (synth.C2, 5000, 30000)])
def test_nll_and_gradient_match_oracle(prec, wl, n_ev, n_nm):
    prob = make_problem(wl, n_ev, n_nm, seed=wl.index)
    ctx = prob.context(_prec(prec))
    tol = (FP64_NLL, FP64_G) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kkk_narrow_phi(prec):
    """The paper's decay (Sec. 4): D+ -> K- K+ K+ with 40 knots and the narrow phi(1020)."""
    wl = synth.KKK
    prob = make_problem(wl, 5000, 30000, seed=6)
    ctx = prob.context(_prec(prec))
    tol = (FP64_NLL, FP64_G) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol, cancelling=(prec == "mixed"))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_cells_full_tiles_and_ragged_tails(prec):
    """Five knots: cells hold thousands of points, so tiles are full with one ragged tail per cell."""
    wl = synth.C2
    kn = synth.uniform_knots(wl.decay, 5)
    prob = make_problem(wl, 20000, 50000, seed=7, knots=kn)
    ctx = prob.context(_prec(prec))
    tol = (FP64_NLL, FP64_G) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_histogram_efficiency_lookup(prec):
    """Efficiency from a 200x200 table, looked up on the device for events and normalisation points."""
    wl = synth.C3
    prob = make_problem(wl, 4000, 20000, seed=3)
    ctx = prob.context(_prec(prec), table_mode=True)
    tol = (FP64_NLL, FP64_G) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mass_and_width_gradient(prec):
    """Shapes floated: resonance amplitudes and their analytic mass/width derivatives on the fly,
    against the oracle's five-point differences."""
    wl = synth.C4
    prob = make_problem(wl, 3000, 20000, seed=4)
    ctx = prob.context(_prec(prec))
    ctx.set_fixed(wl.fixed())
    tol = (FP64_NLL, 1e-7) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol, shapes=True)


# the largest model the library takes: 128 knots and 4 resonances (one of them spin 0); its
# per-evaluation table no longer fits the kernel arguments in either precision
MAX_MODEL = synth.Workload("max_model", 9, "fp64", 2000, 12000, 128,
                           (synth.RHO770, synth.F2_1270, synth.RHO1450, synth.F0_980), "poly", float_shapes=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shapes", [False, True])
def test_largest_model(prec, shapes):
    prob = make_problem(MAX_MODEL, MAX_MODEL.n_events, MAX_MODEL.n_norm, seed=9)
    ctx = prob.context(_prec(prec))
    if shapes:
        ctx.set_fixed(MAX_MODEL.fixed())
        tol = (FP64_NLL, 1e-7) if prec == "fp64" else (MIX_NLL, MIX_G)
    else:
        tol = (FP64_NLL, FP64_G) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol, shapes=shapes)


# a spline S-wave alone (no resonances): the whole amplitude is the spline
SWAVE_ONLY = synth.Workload("swave_only", 10, "fp64", 3000, 20000, 30, (), "flat")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_spline_swave_without_resonances(prec):
    prob = make_problem(SWAVE_ONLY, SWAVE_ONLY.n_events, SWAVE_ONLY.n_norm, seed=10)
    ctx = prob.context(_prec(prec))
    tol = (FP64_NLL, FP64_G) if prec == "fp64" else (MIX_NLL, MIX_G)
    _check(prob, ctx, *tol)
    # the constant S-wave (every knot 1, phase 0) has |A|^2 = 4 everywhere: -2 ln L = 2 n ln(sum w)
    th = np.zeros(2 * SWAVE_ONLY.n_knots)
    th[0::2] = 1.0
    v, _ = ctx.eval(th)
    n = SWAVE_ONLY.n_events
    expect = -2.0 * n * np.log(4.0) + 2.0 * n * np.log(4.0 * np.sum(prob.norm[2]))
    assert abs(v - expect) <= (1e-10 if prec == "fp64" else 1e-6) * abs(expect) + 1e-9 * n, (v, expect)
    ctx.close()


def test_empty_and_oversized_inputs_are_rejected():
    from paper_1703_03284_amd import MipwaError, context_for
    wl = synth.C1
    ctx = context_for(wl.decay, wl.knots(), wl.resonances)
    for call in (lambda: ctx.load_events(np.array([]), np.array([])),
                 lambda: ctx.load_norm(np.array([]), np.array([]), np.array([]))):
        with pytest.raises(MipwaError) as e:
            call()
        assert e.value.status == -1
    ctx.close()
    with pytest.raises(MipwaError) as e:
        context_for(wl.decay, synth.uniform_knots(wl.decay, 129), wl.resonances)
    assert e.value.status == -1
    with pytest.raises(MipwaError) as e:
        context_for(wl.decay, wl.knots(), wl.resonances + (synth.RHO1450, synth.F0_980, synth.F0_1370))
    assert e.value.status == -1


def test_mass_width_gradient_vs_finite_differences():
    """FP64 analytic adjoint vs central differences (h = 1e-6) of the library's own FP64 -2 ln L."""
    wl = synth.C4
    prob = make_problem(wl, 2000, 10000, seed=5)
    ctx = prob.context(_prec("fp64"))
    ctx.set_fixed(wl.fixed())
    _, g = ctx.eval(prob.theta)
    N, R = wl.n_knots, wl.n_res
    for p in list(range(2 * N + 2 * R, 2 * N + 4 * R)) + [0, 1, 2 * N + 2, 2 * N + 3]:
        tp, tm = prob.theta.copy(), prob.theta.copy()
        tp[p] += 1e-6
        tm[p] -= 1e-6
        fd = (ctx.eval(tp)[0] - ctx.eval(tm)[0]) / 2e-6
        assert abs(fd - g[p]) <= 1e-4 * max(1.0, abs(g[p])) + 2e-5 * np.abs(g).max(), (p, fd, g[p])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_consecutive_evaluations_see_their_own_parameters(prec):
    """Back-to-back evaluations on one context, each at new knot, coefficient and shape values.  The
    FP64 tables of 50 knots and three floated resonances exceed the kernel-argument space and go up
    through device memory; the mixed ones travel in the arguments."""
    wl = synth.C4
    prob = make_problem(wl, 2000, 10000, seed=12)
    ctx = prob.context(_prec(prec))
    ctx.set_fixed(wl.fixed())
    tol = FP64_NLL if prec == "fp64" else MIX_NLL
    rng = np.random.Generator(np.random.PCG64(77))
    N, R = wl.n_knots, wl.n_res
    for k in range(4):
        th = prob.theta.copy()
        th[:2 * N + 2 * R] *= 1.0 + 0.01 * rng.standard_normal(2 * N + 2 * R)
        th[2 * N + 2 * R::2] += 1e-3 * k          # masses
        th[2 * N + 2 * R + 1::2] *= 1.0 + 0.01 * k  # widths
        v, _ = ctx.eval(th)
        v_o, _ = prob.oracle(theta=th)
        assert rel(v, v_o) <= tol, (k, v, v_o)


def test_first_evaluation_of_a_new_context_is_its_own():
    """A context created after another of the same size was destroyed returns its own results on its
    first evaluation (its pinned result buffer may reuse the old one's memory)."""
    wl = synth.C1
    a = make_problem(wl, 2000, 10000, seed=21)
    b = make_problem(wl, 2500, 10000, seed=22)
    for _ in range(2):
        ctx = a.context(_prec("mixed"))
        ctx.eval()
        ctx.close()
    ctx = b.context(_prec("mixed"))
    v, _ = ctx.eval()
    assert rel(v, b.oracle()[0]) <= MIX_NLL


def test_cache_rebuilt_when_shapes_change():
    wl = synth.C2
    prob = make_problem(wl, 2000, 10000, seed=8)
    ctx = prob.context(_prec("fp64"))
    ctx.eval()
    th = prob.theta.copy()
    th[-2] *= 1.05   # a width
    th[-3] += 0.01   # a mass
    v, _ = ctx.eval(th)
    v_o, _ = prob.oracle(theta=th)
    assert rel(v, v_o) <= FP64_NLL


def test_deterministic_bitwise():
    prob = make_problem(synth.C2, 5000, 30000, seed=9)
    ctx = prob.context(_prec("mixed"))
    a = ctx.eval()
    b = ctx.eval()
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_single_event_single_point_and_knot_positions():
    wl = synth.C1
    kn = wl.knots()
    # points sitting exactly on knots, plus the degenerate one-point sets
    for ev, nm in [((np.array([0.61]), np.array([1.42])), (np.array([1.1]), np.array([0.95]))),
                   ((kn[[3, 5, 7]], kn[[9, 6, 8]]), (kn[[2, 4]], kn[[10, 12]]))]:
        prob = make_problem(wl, 10, 10, seed=1)
        prob.events = ev
        prob.norm = (nm[0], nm[1], np.full(len(nm[0]), 0.37))
        ctx = prob.context(_prec("fp64"))
        v_o, g_o = prob.oracle()
        v, g = ctx.eval()
        assert rel(v, v_o) <= FP64_NLL
        n_ck = 2 * wl.n_knots + 2 * wl.n_res
        assert np.abs(g[:n_ck] - g_o[:n_ck]).max() <= FP64_G * np.abs(g_o[:n_ck]).max() + 1e-12


def test_errors_are_reported_not_crashed():
    from paper_1703_03284_amd import MipwaError, context_for
    wl = synth.C1
    ctx = context_for(wl.decay, wl.knots(), wl.resonances)
    with pytest.raises(MipwaError) as e:
        ctx.eval(wl.truth())
    assert e.value.status == -4   # E_STATE: nothing loaded
    with pytest.raises(MipwaError) as e:
        ctx.load_events(np.array([0.01]), np.array([0.02]))
    assert e.value.status == -1   # outside the Dalitz region
    with pytest.raises(MipwaError) as e:
        ctx.set_params(np.zeros(3))
    assert e.value.status == -1
    th = wl.truth()
    th[-1] = -0.1
    with pytest.raises(MipwaError):
        ctx.set_params(th)
    # |A|^2 = 0 at every event -> -2 ln L = +inf, reported as E_DOMAIN
    prob = make_problem(wl, 100, 1000, seed=2)
    c2 = prob.context(_prec("fp64"))
    z = prob.theta.copy()
    z[:2 * wl.n_knots + 2 * wl.n_res:2] = 0.0
    with pytest.raises(MipwaError) as e:
        c2.eval(z)
    assert e.value.status == -5
    assert c2.eval(z, raise_domain=False)[0] == float("inf")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_integrals_and_fit_fractions(prec):
    prob = make_problem(synth.C2, 100, 40000, seed=11)
    ctx = prob.context(_prec(prec))
    tol = 1e-10 if prec == "fp64" else 1e-6
    for with_eff in (True, False):
        nm = prob.oracle_norm() if with_eff else prob.norm
        I_o = L.integrals(prob.model, prob.theta, nm)
        I = ctx.integrals(with_eff=with_eff)
        assert np.abs(I - I_o).max() <= tol * np.abs(I_o).max()
        if with_eff:
            # the component integrals recombine to the normalisation integral of the likelihood:
            # I = c^H Ibar c (c_0 = 1), against the oracle's direct sum of w eps |A|^2
            c = L.coefficient_vector(prob.model, prob.theta)
            I_tot = float(np.real(np.conj(c) @ I.T @ c))
            I_dir = L.norm_integral(prob.model, prob.theta, nm)
            assert abs(I_tot - I_dir) <= tol * I_dir, (I_tot, I_dir)
    ff = ctx.fit_fractions()
    ff_o = L.fit_fractions(prob.model, prob.theta, L.integrals(prob.model, prob.theta, prob.norm))
    assert np.abs(ff - ff_o).max() <= 10 * tol
    assert abs(ff.sum() - 1.0) < 1e-12


def test_generator_draw_for_draw():
    wl = synth.C1
    prob = make_problem(wl, 10, 10, seed=0)
    th = wl.truth()
    fmax = 1.5 * OG.density_max(prob.model, th, 77 + 1000, 50_000)
    s12_o, s13_o, exc_o = OG.accept_reject(prob.model, th, 3000, seed=77, fmax=fmax)
    ctx = prob.context(_prec("fp64"))
    s12, s13, exc, ncand = ctx.generate(th, 3000, seed=77, fmax=fmax)
    assert exc == exc_o
    assert np.array_equal(s12, s12_o) and np.array_equal(s13, s13_o)
    assert ctx.density_max(th, 77 + 1000, 50_000) == pytest.approx(fmax / 1.5, rel=1e-12)
