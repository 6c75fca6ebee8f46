"""Toy-fit serving: continuous batching, admission by HBM footprint, isolation between jobs."""
import numpy as np
import pytest

import synth
from oracle import generate as OG
from oracle import kinematics as K
from tests.conftest import oracle_model

pytestmark = pytest.mark.gpu


def _toy(n, n_knots, seed, wl=synth.C1):
    kn = synth.uniform_knots(wl.decay, n_knots)
    truth = synth.truth_theta(n_knots, wl.resonances, seed)
    m = oracle_model(wl, knots=kn)
    s12, s13, _ = OG.toy(m, truth, n, seed=seed, n_probe=100_000)
    start = synth.perturb_theta(truth, n_knots, wl.n_res, seed + 7)
    return kn, truth, start, s12, s13


@pytest.fixture(scope="module")
def norm():
    wl = synth.C1
    s12, s13 = synth.uniform_phase_space(wl.decay, 100_000, 503)
    area = K.area(oracle_model(wl))
    return s12, s13, np.full(len(s12), area / len(s12))


@pytest.fixture(scope="module")
def jobs():
    return {"A": _toy(4000, 20, 11), "B": _toy(8000, 30, 12), "C": _toy(2500, 20, 13), "D": _toy(3000, 40, 14)}


def _server(norm, precision="mixed", budget=0):
    from paper_1703_03284_amd import FP64, MIXED, Server
    s = Server(MIXED if precision == "mixed" else FP64, hbm_budget_bytes=budget)
    s.set_norm(*norm)
    return s


def _submit(srv, job, **kw):
    wl = synth.C1
    kn, _, start, s12, s13 = job
    return srv.submit(wl.decay, kn, wl.resonances, s12, s13, start, **kw)


def test_borrowed_events_give_the_copied_result(norm, jobs):
    # the same jobs submitted with copies and with lent arrays (read by the server when they load):
    # bitwise the same fits, the lent arrays untouched, and released once the final result is read
    with _server(norm) as s1:
        ref = [s1.wait(_submit(s1, jobs[k])) for k in ("A", "B")]
    lent = {k: (jobs[k][3].copy(), jobs[k][4].copy()) for k in ("A", "B")}
    with _server(norm) as s2:
        ids = []
        for k in ("A", "B"):
            kn, _, start, _, _ = jobs[k]
            wl = synth.C1
            ids.append(s2.submit(wl.decay, kn, wl.resonances, lent[k][0], lent[k][1], start, copy=False))
        assert set(s2._borrowed) == set(ids)
        got = [s2.wait(i) for i in ids]
        assert s2._borrowed == {}
    for r, g in zip(ref, got):
        assert r["status"] == 0 and g["status"] == 0
        assert np.array_equal(r["theta"], g["theta"]) and r["nll"] == g["nll"] and r["n_eval"] == g["n_eval"]
    for k in ("A", "B"):
        assert np.array_equal(lent[k][0], jobs[k][3]) and np.array_equal(lent[k][1], jobs[k][4])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_result_alone_equals_result_in_the_mix(norm, jobs, precision):
    with _server(norm, precision) as s1:
        a = s1.wait(_submit(s1, jobs["A"]))
    with _server(norm, precision) as s2:
        ids = [_submit(s2, jobs[k]) for k in ("B", "A", "C", "D")]
        res = [s2.wait(i) for i in ids]
        st = s2.stats()
    a_mix = res[1]
    assert a["status"] == 0 and a_mix["status"] == 0
    assert np.array_equal(a["theta"], a_mix["theta"])
    assert a["nll"] == a_mix["nll"] and a["n_eval"] == a_mix["n_eval"]
    assert st["n_done"] == 4 and st["mean_batch"] > 1.0


def test_jobs_with_the_same_shapes_share_moments_without_changing_results(norm, jobs):
    # held shapes at their table values: two jobs with the same knots use one set of normalisation
    # moments, formed by whichever loads first; a third job with the same knots but shapes of its own
    # gets its own.  The first job's fit is bitwise the one it gets alone.
    wl = synth.C1
    held = {}
    for k in ("A", "C"):
        kn, truth, _, s12, s13 = jobs[k]
        held[k] = (kn, truth, synth.fit_start(truth, len(kn), wl.n_res, 100 + ord(k)), s12, s13)
    with _server(norm) as s1:
        alone = s1.wait(_submit(s1, held["A"]))
    with _server(norm) as s2:
        ids = [_submit(s2, held["C"]), _submit(s2, jobs["C"]), _submit(s2, held["A"])]
        res = [s2.wait(i) for i in ids]
    assert alone["status"] == 0 and all(r["status"] == 0 for r in res)
    assert np.array_equal(alone["theta"], res[2]["theta"])
    assert alone["nll"] == res[2]["nll"] and alone["n_eval"] == res[2]["n_eval"]
    # the held parameters stay where the start put them (the reference phase up to the fold's rounding)
    fx = synth.fixed_mask(len(held["A"][0]), wl.n_res).astype(bool)
    assert np.allclose(res[2]["theta"][fx], held["A"][1][fx], rtol=0, atol=1e-12)


def test_serving_fit_agrees_with_single_context_fit(norm, jobs):
    from paper_1703_03284_amd import FP64, context_for
    wl = synth.C1
    kn, _, start, s12, s13 = jobs["A"]
    with _server(norm, "fp64") as srv:
        r = srv.wait(_submit(srv, jobs["A"], tol_edm=1e-8))
    ctx = context_for(wl.decay, kn, wl.resonances, FP64)
    ctx.load_events(s12, s13)
    ctx.load_norm(*norm)
    ref = ctx.fit(start, fixed=synth.fixed_mask(20, wl.n_res), tol_edm=1e-8)
    free = np.flatnonzero(synth.fixed_mask(20, wl.n_res) == 0)
    d = r["theta"] - ref.theta
    npair = 20 + wl.n_res
    d[1:2 * npair:2] = np.angle(np.exp(1j * d[1:2 * npair:2]))
    assert (np.abs(d[free]) / ref.sigma[free]).max() < 0.01


def test_admission_under_a_small_budget(norm, jobs):
    # room for the normalisation sets and about one job at a time
    with _server(norm, "mixed", budget=48 << 20) as srv:
        ids = [_submit(srv, jobs[k]) for k in ("A", "B", "C", "D")]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert all(r["status"] == 0 for r in res)
    assert st["n_done"] == 4


def test_cancel_leaves_other_jobs_alone(norm, jobs):
    with _server(norm, "mixed") as ref_srv:
        ref = ref_srv.wait(_submit(ref_srv, jobs["C"]))
    with _server(norm, "mixed") as srv:
        a = _submit(srv, jobs["A"])
        b = _submit(srv, jobs["B"])
        c = _submit(srv, jobs["C"])
        srv.cancel(b)
        ra, rb, rc = srv.wait(a), srv.wait(b), srv.wait(c)
    assert rb["status"] == -7
    assert ra["status"] == 0 and rc["status"] == 0
    assert np.array_equal(rc["theta"], ref["theta"])


def test_invalid_submissions_are_rejected(norm, jobs):
    from paper_1703_03284_amd import MipwaError
    wl = synth.C1
    kn, _, start, s12, s13 = jobs["A"]
    with _server(norm, "mixed") as srv:
        fx = synth.fixed_mask(20, wl.n_res, float_shapes=True)
        with pytest.raises(MipwaError):
            srv.submit(wl.decay, kn, wl.resonances, s12, s13, start, fixed=fx)
        bad = start.copy()
        bad[-1] = -1.0
        with pytest.raises(MipwaError):
            srv.submit(wl.decay, kn, wl.resonances, s12, s13, bad)
        ok = srv.wait(_submit(srv, jobs["C"]))
        assert ok["status"] == 0


@pytest.mark.parametrize("copy", [True, False], ids=["copied", "lent"])
def test_cancellation_at_any_point_and_teardown_with_work_in_flight(norm, jobs, copy):
    """Many jobs, cancelled at staggered times (queued, waiting for a loader stream, loading, between
    steps or inside one), then the server closed while the rest are still running: every wait
    returns, the cancelled ones as E_CANCELLED, the others converged or cancelled by the teardown,
    and an untouched job's result is the one it gets alone; with the events copied or lent."""
    import time
    with _server(norm, "mixed") as ref_srv:
        ref = ref_srv.wait(_submit(ref_srv, jobs["D"]))
    srv = _server(norm, "mixed")
    keys = ["A", "B", "C"] * 8
    ids = [_submit(srv, jobs[k], copy=copy) for k in keys]
    keep = _submit(srv, jobs["D"], copy=copy)
    for k, j in enumerate(ids[::2]):
        time.sleep(0.002 * (k % 4))
        srv.cancel(j)
    res_keep = srv.wait(keep)
    assert res_keep["status"] == 0
    assert np.array_equal(res_keep["theta"], ref["theta"])
    for j in ids[::2]:
        assert srv.wait(j)["status"] in (-7, 0, -6)  # a job may finish before its cancel lands
    for k in ("A", "B"):
        _submit(srv, jobs[k], copy=copy)
    srv.close()  # jobs still queued or running are cancelled; nothing hangs or faults
