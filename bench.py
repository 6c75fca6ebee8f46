"""Benchmark: -2 ln L + gradient evaluations per second on one MI355X.

Workload (default): D+ -> pi- pi+ pi+, 10M toy events generated on the device by accept-reject at
the truth parameters, 10M uniform phase-space normalisation points, 50 S-wave knots, rho(770) and
f2(1270), efficiency from a 200x200 FP32 table; mixed precision (FP32 streams and amplitudes, FP64
accumulation and finish).  One step = one full evaluation (parameter upload, spline setup, the
streaming forward+adjoint kernel over both point sets, reduction, FP64 finish, result readback).
The plain FP64 GPU path is timed on the same workload and reported beside it; the FP64 oracle evaluates
the same inputs on the host's cores (cpu_baseline) and the mixed-precision results are stated against
it (vs_oracle).

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cpu] [--no-fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_PERIOD = 4  # every 4th timed evaluation records device-time events


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_point(precision_bytes: int, kind: str) -> int:
    """Bytes the method must read per point and evaluation: its two coordinates (t12, t13) and, for a
    normalisation point, its weight x efficiency."""
    return 2 * precision_bytes + (precision_bytes if kind == "norm" else 0)


def stream_bytes_per_point(precision_bytes: int, n_res: int, kind: str) -> int:
    """Bytes the streaming kernel reads per point by design: the algorithmic bytes plus the cached
    symmetrised amplitude of each resonance (one complex number)."""
    return algorithmic_bytes_per_point(precision_bytes, kind) + 2 * n_res * precision_bytes


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_eval_mixed_10M_traffic.md")
TRAFFIC_PROFILE_FP64 = os.path.join(ROOT, "profiles", "k_eval_fp64_10M_kernel_trace_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1703_03284_amd", "csrc", "kernels.hip")


def recorded_traffic(path):
    """HBM bytes per launch of the streaming kernel from a committed counter summary (FETCH_SIZE +
    WRITE_SIZE, each scaled by a 1 GiB copy), or None once the kernel source differs from the one
    the counters were taken on."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith(" "))
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("Kernel source sha256 (csrc/kernels.hip)", "").strip() != src or \
            "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def build_inputs(wl, n_events, n_norm):
    import synth
    from paper_1703_03284_amd import FP64, context_for
    d = wl.decay
    table = synth.efficiency_histogram(synth.PolyEfficiency.seeded(d, wl.seed("eff"))) \
        if wl.efficiency == "hist" else None
    truth = wl.truth()
    t0 = time.time()
    gen = context_for(d, wl.knots(), wl.resonances, FP64)
    if table is not None:
        gen.set_eff_table(table, d.smin, d.smax)
    ev12, ev13, fmax = gen.toy(truth, n_events, wl.seed("events"))
    gen.close()
    log(f"[bench] generated {n_events} toy events on the device in {time.time() - t0:.1f}s (fmax={fmax:.4g})")
    t0 = time.time()
    n12, n13 = synth.uniform_phase_space(d, n_norm, wl.seed("norm"))
    area = synth.region_area_mc(d, 1 << 22, 5)  # only used as a constant weight scale
    w = np.full(n_norm, area / n_norm)
    log(f"[bench] normalisation points in {time.time() - t0:.1f}s")
    return table, (ev12, ev13), (n12, n13, w)


def time_gpu(wl, precision, table, events, norm, steps, warmup, blocks=0, waves=0, qform=False):
    from paper_1703_03284_amd import NORM_QFORM, context_for
    d = wl.decay
    ctx = context_for(d, wl.knots(), wl.resonances, precision)
    if blocks or waves:
        ctx.set_launch(blocks, waves)
    if qform:
        ctx.set_norm_mode(NORM_QFORM)
    if wl.float_shapes:
        ctx.set_fixed(wl.fixed())   # masses and widths floated: resonances on the fly every evaluation
    if table is not None:
        ctx.set_eff_table(table, d.smin, d.smax)
    t0 = time.time()
    ctx.load_events(*events)
    ctx.load_norm(*norm)
    log(f"[bench] loaded {len(events[0])} + {len(norm[0])} points in {time.time() - t0:.1f}s")
    th0 = wl.start()
    rng = np.random.Generator(np.random.PCG64(12345))
    n_shape = 0 if wl.float_shapes else 4 * wl.n_res
    for _ in range(warmup):
        ctx.eval(th0)
    thetas = []
    for _ in range(steps):
        th = th0.copy()
        th[:len(th) - n_shape] += 1e-9 * rng.standard_normal(len(th) - n_shape)  # no result can be reused
        thetas.append(th)
    # HIP events on the evaluation stream, accumulated by the library: every TIMING_PERIOD-th evaluation
    # of the timed loop records them, alternately around the whole evaluation and around the
    # streaming kernel (each recorded pair adds device time to its evaluation)
    ctx.set_timing(TIMING_PERIOD)
    t0 = time.perf_counter()
    for th in thetas:
        ctx.eval(th)
    wall = time.perf_counter() - t0
    n_timed, dev_ms, stream_ms = ctx.timing_stats()
    ctx.set_timing(0)
    nll, grad = ctx.eval(th0)
    ff = None if wl.float_shapes else ctx.fit_fractions(th0)
    ctx.close()
    assert n_timed == -(-steps // TIMING_PERIOD)
    return {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "value": steps / wall,
            "dev_ms": dev_ms, "stream_kernel_ms": stream_ms, "nll": nll, "grad": grad, "ff": ff}


def oracle_leg(wl, table, events, norm, mixed, reps=1):
    """The FP64 oracle on the headline inputs themselves (the same toy events, normalisation points
    and efficiency table as the GPU run), split in 1M-point chunks over worker processes on the host's
    cores: one evaluation that also warms the workers up, then `reps` timed evaluations (the CPU
    baseline).  Compares the mixed-precision library's -2 ln L, gradient and fit fractions at the same
    point with the oracle's; the gradient error is also weighted by the errors sigma_p of a fit of this
    sample, taken from the expected information (oracle, 200k-point subsample)."""
    from threadpoolctl import threadpool_limits
    from oracle import Model, Res
    from oracle import likelihood as L
    from oracle.pool import OraclePool
    d = wl.decay
    m = Model(d.M, d.m1, d.m2, d.m3, d.rD, tuple(wl.knots()),
              tuple(Res(r.spin, r.mass, r.width, r.radius) for r in wl.resonances))
    th = wl.start()
    n12, n13, w = norm
    e_ev = L.hist_lookup(table, d.smin, d.smax, *events) if table is not None else np.ones(len(events[0]))
    e_nm = L.hist_lookup(table, d.smin, d.smax, n12, n13) if table is not None else np.ones(len(n12))
    t0 = time.perf_counter()
    pool = OraclePool(m, events, (n12, n13, w * e_nm), float(np.sum(np.log(e_ev))), w_plain=w)
    try:
        log(f"[bench] oracle: {pool.workers} worker processes, arrays mapped in {time.perf_counter() - t0:.1f}s")
        v_o, g_o = pool.nll_and_grad(th)
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            pool.nll_and_grad(th)
            times.append(time.perf_counter() - t0)
        t_all = float(np.median(times))
        free = np.flatnonzero(wl.fixed() == 0)
        sigma = pool.expected_sigma(th, free, 200_000)
        ff_o = L.fit_fractions(m, th, pool.integrals(th))
        workers = pool.workers
    finally:
        pool.close()
    # one core: the same oracle on one 1M + 1M chunk in this process, scaled to the full inputs
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        L.point_sums(m, th, events[0][:1_000_000], events[1][:1_000_000], None, False)
        L.point_sums(m, th, n12[:1_000_000], n13[:1_000_000], (w * e_nm)[:1_000_000], False)
        t1 = (time.perf_counter() - t0) * (len(events[0]) + len(n12)) / 2_000_000
    n_ck = 2 * wl.n_knots + 2 * wl.n_res
    v, g, ff = mixed["nll"], mixed["grad"], mixed["ff"]
    dg = np.abs(g[:n_ck] - g_o[:n_ck])
    vs = {"point": "the start point of the fits (truth perturbed)",
          "nll": v, "nll_oracle": v_o, "nll_abs": abs(v - v_o), "nll_rel": abs(v - v_o) / abs(v_o),
          "grad_rel_inf": float(dg.max() / np.abs(g_o[:n_ck]).max()),
          "grad_sigma_weighted": float(np.max(dg[free[free < n_ck]] * sigma[free[free < n_ck]])),
          "ff_abs_max": float(np.abs(np.diag(ff) - np.diag(ff_o)).max()),
          "ff_oracle": [float(x) for x in np.diag(ff_o)]}
    cpu = {"value": 1.0 / t_all, "unit": "evals/s", "cores": workers, "kind": "oracle",
           "sample": f"the full headline inputs ({len(events[0])} toy events + {len(n12)} normalisation points, "
                     f"the same arrays as the GPU run), -2 ln L + knot and coefficient gradient, split in 1M-point "
                     f"chunks over {workers} worker processes, median of {reps} after one warm-up evaluation; "
                     f"{t_all:.2f} s per evaluation",
           "one_core": {"value": 1.0 / t1, "cores": 1, "seconds_per_eval": t1,
                        "how": "one 1M + 1M chunk in one process, scaled to the full inputs"}}
    return cpu, vs


def headline_fit_mixed_vs_fp64(wl, table, events, norm):
    """The headline sample fitted in mixed precision and in FP64 by the library, from the same start:
    the largest |d theta| / sigma over the floated parameters (sigma from the FP64 fit's Hessian).  An
    oracle fit of 10M + 10M points would take minutes; the FP64 path stands in for it (it agrees with
    the oracle to 1e-10 in -2 ln L and 1e-8 in the gradient at this size)."""
    from paper_1703_03284_amd import FP64, MIXED, context_for
    d = wl.decay
    res = {}
    for name, prec in (("fp64", FP64), ("mixed", MIXED)):
        ctx = context_for(d, wl.knots(), wl.resonances, prec)
        if table is not None:
            ctx.set_eff_table(table, d.smin, d.smax)
        ctx.load_events(*events)
        ctx.load_norm(*norm)
        t0 = time.perf_counter()
        res[name] = (ctx.fit(wl.start(), fixed=wl.fixed(), tol_edm=1e-6, raise_noconv=False),
                     time.perf_counter() - t0)
        ctx.close()
    (f64, t64), (f32, t32) = res["fp64"], res["mixed"]
    free = np.flatnonzero(wl.fixed() == 0)
    dth = f32.theta - f64.theta
    npair = wl.n_knots + wl.n_res
    dth[1:2 * npair:2] = np.angle(np.exp(1j * dth[1:2 * npair:2]))
    ratio = f32.sigma[free] / f64.sigma[free]
    return {"fit_theta_max_sigma_vs_fp64": float(np.max(np.abs(dth[free]) / f64.sigma[free])),
            "sigma_ratio_min": float(ratio.min()), "sigma_ratio_max": float(ratio.max()),
            "nll_mixed_minus_fp64": f32.nll - f64.nll, "status": [f64.status, f32.status],
            "evals": [f64.n_eval, f32.n_eval], "fit_s": [round(t64, 3), round(t32, 3)],
            "floated": int(len(free))}


def small_fit_vs_oracle():
    """The 10k-event fit workload fitted by the library in mixed precision and by the oracle (scipy
    BFGS, V = 2 H^-1) from the same start on the same toy: the largest |d theta| / sigma over the
    floated parameters, the spread of the error ratio and of the fit-fraction difference."""
    import synth
    from oracle import fit as OF
    from oracle import generate as OG
    from oracle import kinematics as K
    from oracle import likelihood as L
    from oracle import Model, Res
    from paper_1703_03284_amd import MIXED, context_for
    wl = synth.C1
    d = wl.decay
    m = Model(d.M, d.m1, d.m2, d.m3, d.rD, tuple(wl.knots()),
              tuple(Res(r.spin, r.mass, r.width, r.radius) for r in wl.resonances))
    s12, s13, _ = OG.toy(m, wl.truth(), wl.n_events, seed=wl.seed("events"), n_probe=200_000)
    n12, n13 = synth.uniform_phase_space(d, wl.n_norm, wl.seed("norm"))
    norm = (n12, n13, np.full(len(n12), K.area(m) / len(n12)))
    t0 = time.perf_counter()
    ref = OF.fit(m, wl.start(), (s12, s13), norm, wl.fixed(), gtol=1e-6)
    t_oracle = time.perf_counter() - t0
    ctx = context_for(d, wl.knots(), wl.resonances, MIXED)
    ctx.load_events(s12, s13)
    ctx.load_norm(*norm)
    t0 = time.perf_counter()
    res = ctx.fit(wl.start(), fixed=wl.fixed(), tol_edm=1e-8)
    t_lib = time.perf_counter() - t0
    ff = np.diag(ctx.fit_fractions(res.theta))
    ctx.close()
    free = np.flatnonzero(wl.fixed() == 0)
    dth = res.theta - ref["theta"]
    npair = wl.n_knots + wl.n_res
    dth[1:2 * npair:2] = np.angle(np.exp(1j * dth[1:2 * npair:2]))
    ratio = res.sigma[free] / ref["sigma"][free]
    ff_o = np.diag(L.fit_fractions(m, ref["theta"], L.integrals(m, ref["theta"], norm)))
    return {"workload": f"D+->pi-pi+pi+ {wl.n_events} toy events + {wl.n_norm} normalisation points, "
                        f"{wl.n_knots} knots, rho(770)+f2(1270), {len(free)} floated parameters",
            "precision": "mixed", "fit_theta_max_sigma": float(np.max(np.abs(dth[free]) / ref["sigma"][free])),
            "sigma_ratio_min": float(ratio.min()), "sigma_ratio_max": float(ratio.max()),
            "ff_abs_max": float(np.abs(ff - ff_o).max()), "nll_abs": abs(res.nll - ref["nll"]),
            "library_fit_s": round(t_lib, 3), "oracle_fit_s": round(t_oracle, 1), "evals": res.n_eval,
            "status": res.status}


def serving(n_jobs, precision, rate_factor=0.8, log_every=32, borrow=True):
    """Toy-fit serving: n_jobs fits (event counts log-uniform in [1e4, 5e6], knots in {20,30,40,50},
    rho(770)+f2(1270), shapes held at their table values) against one shared 2M-point normalisation
    sample.  Run 1 submits every job at t=0 (capacity); run 2 submits them at Poisson arrival times
    with rate rate_factor x capacity and reports fits/s and p50/p99 time-to-fit.  borrow: the jobs'
    event arrays are lent to the server (read when each job loads) instead of copied at submission."""
    import synth
    from paper_1703_03284_amd import FP64, Server, context_for
    wl = synth.C1
    d = wl.decay
    specs = synth.serving_jobs(n_jobs)
    n12, n13 = synth.uniform_phase_space(d, 2_000_000, synth.SERVE_NORM_SEED)
    w = np.full(len(n12), synth.region_area_mc(d, 1 << 22, 5) / len(n12))
    gens = {}
    payload = []
    t0 = time.time()
    for i, (n, N, seed) in enumerate(specs):
        if N not in gens:
            gens[N] = context_for(d, synth.uniform_knots(d, N), wl.resonances, FP64)
        truth = synth.truth_theta(N, wl.resonances, seed)
        s12, s13, _ = gens[N].toy(truth, n, seed, n_probe=200_000)
        payload.append((synth.uniform_knots(d, N), s12, s13, synth.fit_start(truth, N, wl.n_res, seed + 7)))
    for g in gens.values():
        g.close()
    n_events = sum(len(p[1]) for p in payload)
    log(f"[bench] serving: generated {n_events} toy events for {n_jobs} jobs in {time.time() - t0:.1f}s")

    def run(arrivals):
        srv = Server(precision)
        srv.set_norm(n12, n13, w)
        ids = []
        start = time.perf_counter()
        for i, (kn, s12, s13, th0) in enumerate(payload):
            if arrivals is not None:
                delay = arrivals[i] - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
            ids.append(srv.submit(d, kn, wl.resonances, s12, s13, th0, tol_edm=1e-4, copy=not borrow))
        t_submit = time.perf_counter() - start
        res = []
        for k, j in enumerate(ids):
            res.append(srv.wait(j))
            if (k + 1) % log_every == 0:
                log(f"[bench] serving: {k + 1}/{len(ids)} fits done")
        wall = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        n_ok = sum(1 for r in res if r["status"] == 0)
        n_noconv = sum(1 for r in res if r["status"] == -6)
        log(f"[bench] serving: submissions took {t_submit:.3f}s of the run's {wall:.3f}s")
        st["submission_s"] = t_submit
        return wall, st, (n_ok, n_noconv), res

    wall0, st0, ok0, _ = run(None)
    capacity = st0["fits_per_s"]
    log(f"[bench] serving capacity run: {st0} wall {wall0:.1f}s")
    rate = rate_factor * capacity
    arrivals = synth.poisson_arrivals(n_jobs, rate, seed=502)
    wall1, st1, ok1, res1 = run(arrivals)
    log(f"[bench] serving Poisson run: {st1} wall {wall1:.1f}s")
    return {"jobs": n_jobs, "events_total": int(n_events), "norm_points": len(n12),
            "capacity_fits_per_s": capacity, "arrival_rate_per_s": rate,
            "fits_per_s": st1["fits_per_s"], "p50_s": st1["p50_s"], "p99_s": st1["p99_s"],
            "mean_batch": st1["mean_batch"], "steps": st1["steps"], "peak_bytes": st1["peak_bytes"],
            "capacity_device_busy": st0["device_busy"], "capacity_step_device_us": 1e6 * st0["step_device_s"],
            "capacity_mean_batch": st0["mean_batch"], "capacity_steps": st0["steps"],
            "capacity_submission_s": st0["submission_s"], "submission": "borrowed" if borrow else "copied",
            "device_busy": st1["device_busy"], "step_device_us": 1e6 * st1["step_device_s"],
            "converged": ok1[0], "not_converged": ok1[1], "tol_edm": 1e-4,
            "mean_evals_per_fit": float(np.mean([r.get("n_eval", 0) for r in res1])),
            "precision": "mixed" if precision == 1 else "fp64"}


def paper_fit(precision_name="fp64"):
    """The paper's fit (Sec. 4) on synthetic input: D+ -> K-K+K+, 40 knots, phi(1020), 100k toy events
    generated on the device at the truth, fitted (BFGS from a perturbed start, Hessian at the end)
    with the normalisation integral on the evenly spaced grid at each spacing of Fig. 2.  Reports the
    fit wall time (the paper's Table 1 times this fit on 2014-era GPUs) and the pulls of the fitted
    knot values against the input (the quantity Fig. 2 plots)."""
    import synth
    from paper_1703_03284_amd import FP64, MIXED, context_for
    wl = synth.KKK
    d = wl.decay
    prec = FP64 if precision_name == "fp64" else MIXED
    truth = wl.truth()
    gen = context_for(d, wl.knots(), wl.resonances, FP64)
    ev12, ev13, _ = gen.toy(truth, wl.n_events, wl.seed("events"))
    gen.close()
    N = wl.n_knots
    out = []
    for h in (0.01, 0.004, 0.001):
        grid = synth.grid_points(d, h)
        ctx = context_for(d, wl.knots(), wl.resonances, prec)
        ctx.load_events(ev12, ev13)
        ctx.load_norm(*grid)
        # the parameters held fixed (the reference coefficient, mass and width) stay at the input
        # values; only the floated ones start perturbed
        fixed = wl.fixed()
        start = np.where(fixed == 1, truth, wl.start())
        t0 = time.perf_counter()
        fit = ctx.fit(start, fixed=fixed, tol_edm=1e-4, hessian=True, raise_noconv=False)
        wall = time.perf_counter() - t0
        ctx.close()
        sig = fit.sigma
        dth = fit.theta - truth
        dth[1:2 * N:2] = np.angle(np.exp(1j * dth[1:2 * N:2]))
        knot = np.arange(2 * N)
        ok = sig[knot] > 0
        pulls = dth[knot][ok] / sig[knot][ok]
        row = {"spacing_GeV2": h, "grid_points": len(grid[0]), "fit_s": round(wall, 3), "evals": fit.n_eval,
               "iterations": fit.n_iter, "status": fit.status, "nll": fit.nll,
               "knot_pull_mean_abs": float(np.mean(np.abs(pulls))), "knot_pull_max_abs": float(np.max(np.abs(pulls))),
               "knot_pull_rms": float(np.sqrt(np.mean(pulls ** 2)))}
        log(f"[bench] paper fit, grid {h}: {row}")
        out.append(row)
    return {"workload": f"D+->K-K+K+ {wl.n_events} toy events, {N} knots, phi(1020), grid normalisation",
            "precision": precision_name, "fits": out}


# Arithmetic of one point with masses and widths floated, counted from the formulas as FP32 vector
# operations (add, multiply, FMA and compare-select count one each) plus transcendentals (reciprocal,
# square root, reciprocal square root, log).  Per pairing of the Breit-Wigner (x, y): the shared
# kinematics (q^2, p^2, sqrt x, q, T_1, T_2) take 23 operations and 3 transcendentals; each resonance
# takes 19 (L = 1) or 22 (L = 2) operations and 3 transcendentals for its value and 19 more for its
# mass and width partials.  Per point: the two spline axes, |A|^2 and the spline adjoint take 36, the
# data seed (log, reciprocal) 5 and 2 transcendentals, the normalisation seed 4; each resonance adds
# 16 for its combination into A and its coefficient, mass and width adjoints.
def otf_ops_per_point(spins, kind):
    pairing = 23 + sum((19 if L == 1 else 22) + 19 for L in spins)
    ops = 2 * pairing + 36 + (5 if kind == "data" else 4) + 16 * len(spins)
    trans = 2 * (3 + 3 * len(spins)) + (2 if kind == "data" else 0)
    return ops, trans


# The vector ALU ceiling without packed FP32 math (the library is compiled without it): 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz lane-operations per second; a transcendental takes four operation slots.
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
TRANS_SLOTS = 4


def shapes_floated(steps, warmup, precision_name):
    """The 5M + 5M workload with every mass and width floated: no resonance cache, the resonances
    and their mass/width partials are evaluated on the fly at every point of every evaluation."""
    import synth
    from paper_1703_03284_amd import FP64, MIXED
    wl = synth.C4
    table, events, norm = build_inputs(wl, wl.n_events, wl.n_norm)
    prec = {"mixed": MIXED, "fp64": FP64}[precision_name]
    r = time_gpu(wl, prec, table, events, norm, steps, warmup)
    log(f"[bench] shapes floated, {precision_name}: {r}")
    return {"workload": f"D+->pi-pi+pi+ {wl.n_events} toy events + {wl.n_norm} uniform normalisation points, "
                        f"{wl.n_knots} knots, rho(770)+f2(1270)+rho(1450) with masses and widths floated",
            "precision": precision_name, "value": r["value"], "unit": "evals/s", "ms_per_step": r["ms_per_step"],
            "device_ms_per_step": r["dev_ms"], "stream_kernel_ms": r["stream_kernel_ms"]}


def smaller_workloads(steps, warmup):
    """The 10k-event fit workload (latency-bound: a few MB per evaluation) and the 1M-event FP64
    workload with the polynomial efficiency per point (208 MB per evaluation, within the 256 MB
    Infinity Cache), both in FP64 as their fits are."""
    import synth
    from paper_1703_03284_amd import FP64, context_for
    out = []
    for wl in (synth.C1, synth.C2):
        d = wl.decay
        pe = synth.PolyEfficiency.seeded(d, wl.seed("eff")) if wl.efficiency == "poly" else None
        gen = context_for(d, wl.knots(), wl.resonances, FP64)
        if pe is not None:
            gen.set_eff_table(synth.efficiency_histogram(pe), d.smin, d.smax)
        ev12, ev13, _ = gen.toy(wl.truth(), wl.n_events, wl.seed("events"))
        gen.close()
        n12, n13 = synth.uniform_phase_space(d, wl.n_norm, wl.seed("norm"))
        w = np.full(wl.n_norm, synth.region_area_mc(d, 1 << 22, 5) / wl.n_norm)
        events = (ev12, ev13) if pe is None else (ev12, ev13, pe(ev12, ev13))
        norm = (n12, n13, w) if pe is None else (n12, n13, w, pe(n12, n13))
        r = time_gpu(wl, FP64, None, events, norm, steps, warmup)
        nbytes = wl.n_events * stream_bytes_per_point(8, wl.n_res, "data") + \
            wl.n_norm * stream_bytes_per_point(8, wl.n_res, "norm")
        out.append({"workload": f"D+->pi-pi+pi+ {wl.n_events} toy events + {wl.n_norm} uniform normalisation points, "
                                f"{wl.n_knots} knots, {wl.n_res} resonances, efficiency {wl.efficiency}",
                    "precision": "fp64", "value": r["value"], "unit": "evals/s", "ms_per_step": r["ms_per_step"],
                    "device_ms_per_step": r["dev_ms"], "stream_kernel_ms": r["stream_kernel_ms"],
                    "bytes_per_launch": nbytes,
                    "achieved_GBs": nbytes / (r["stream_kernel_ms"] * 1e-3) / 1e9})
        log(f"[bench] {out[-1]}")
    return out


def profile_pass(steps, which="headline"):
    """A few evaluations of one workload plus a 1 GiB device copy of known size (counter calibration)."""
    import torch
    import synth
    from paper_1703_03284_amd import FP64, MIXED
    wl = synth.C4 if which == "shapes" else synth.C3
    table, events, norm = build_inputs(wl, wl.n_events, wl.n_norm)
    r = time_gpu(wl, FP64 if which == "fp64" else MIXED, table, events, norm, steps, 2)
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] profile pass: {r}; copy of {a.numel() * 4} bytes x3")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--events", type=int, default=None)
    ap.add_argument("--norm", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-paper-fit", action="store_true")
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=256)
    ap.add_argument("--profile-pass", nargs="?", const="headline", choices=["headline", "shapes", "fp64"])
    ap.add_argument("--no-shapes", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the likelihood would shard "
              "by points with one small all-reduce per evaluation).", file=sys.stderr)
        sys.exit(2)
    if args.profile_pass:
        profile_pass(args.steps, args.profile_pass)
        return
    import synth
    from paper_1703_03284_amd import FP64, MIXED, read_bandwidth
    wl = synth.C3
    n_ev = args.events or wl.n_events
    n_nm = args.norm or wl.n_norm
    table, events, norm = build_inputs(wl, n_ev, n_nm)
    mixed = time_gpu(wl, MIXED, table, events, norm, args.steps, args.warmup, args.blocks, args.waves)
    log(f"[bench] mixed: { {k: v for k, v in mixed.items() if k not in ('grad', 'ff')} }")
    fp64 = None
    if not args.no_fp64:
        fp64 = time_gpu(wl, FP64, table, events, norm, args.steps, args.warmup, args.blocks, args.waves)
        log(f"[bench] fp64: { {k: v for k, v in fp64.items() if k not in ('grad', 'ff')} }")
    ceiling = read_bandwidth(0, 1 << 30, 10)
    log(f"[bench] measured streaming-read ceiling: {ceiling:.0f} GB/s")

    def roof(prec_bytes, kernel_ms, kernel, traffic):
        alg = n_ev * algorithmic_bytes_per_point(prec_bytes, "data") + n_nm * algorithmic_bytes_per_point(prec_bytes, "norm")
        des = n_ev * stream_bytes_per_point(prec_bytes, wl.n_res, "data") + \
            n_nm * stream_bytes_per_point(prec_bytes, wl.n_res, "norm")
        sec = kernel_ms * 1e-3
        r = {"bound": "hbm", "achieved": alg / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": alg / sec / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
             "kernel": kernel, "kernel_ms": kernel_ms, "algorithmic_bytes_per_launch": alg,
             "design_bytes_per_launch": des, "design_achieved": des / sec / 1e9,
             "design_frac": des / sec / 1e9 / HBM_PEAK_GBS,
             "measured_read_ceiling_GBs": ceiling, "design_frac_of_measured_ceiling": des / sec / 1e9 / ceiling}
        if traffic is not None:
            r["traffic_over_algorithmic"] = traffic / alg
            r["traffic_over_design"] = traffic / des
        return r

    full = (n_ev, n_nm) == (wl.n_events, wl.n_norm)
    out = {
        "metric": "NLL+grad evals/sec @10M events (mixed vs FP64 GPU); toy fits/sec + p50/p99",
        "value": mixed["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D+->pi-pi+pi+ {n_ev} toy events + {n_nm} uniform normalisation points, "
                               f"{wl.n_knots} knots, rho(770)+f2(1270), 200x200 efficiency table, mixed precision",
                   "events": n_ev, "norm_points": n_nm, "knots": wl.n_knots, "resonances": wl.n_res,
                   "accumulate": "f64"},
        "device_ms_per_step": mixed["dev_ms"],
        "fp64": None if fp64 is None else {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                                           "device_ms_per_step": fp64["dev_ms"],
                                           "stream_kernel_ms": fp64["stream_kernel_ms"],
                                           "mixed_speedup": mixed["value"] / fp64["value"],
                                           "roofline": roof(8, fp64["stream_kernel_ms"], "k_eval<double,2,false>",
                                                            recorded_traffic(TRAFFIC_PROFILE_FP64) if full else None)},
        "roofline": roof(4, mixed["stream_kernel_ms"], "k_eval<float,2,false>",
                         recorded_traffic(TRAFFIC_PROFILE) if full else None),
    }
    # the same evaluation with the normalisation as a quadratic form over per-cell moments (an
    # algebraic rearrangement beyond the paper; reported beside the headline, not as it)
    qf = time_gpu(wl, MIXED, table, events, norm, args.steps, args.warmup, args.blocks, args.waves, qform=True)
    log(f"[bench] mixed, quadratic-form normalisation: {qf}")
    out["quadratic_form_norm"] = {"value": qf["value"], "ms_per_step": qf["ms_per_step"],
                                  "device_ms_per_step": qf["dev_ms"], "stream_kernel_ms": qf["stream_kernel_ms"],
                                  "nll_minus_point_sweep": qf["nll"] - mixed["nll"]}
    if not args.no_shapes:
        sh = {p: shapes_floated(max(10, args.steps // 4), 3, p) for p in ("mixed", "fp64")}
        spins = [r.spin for r in synth.C4.resonances]
        slots = 0
        for kind, n in (("data", synth.C4.n_events), ("norm", synth.C4.n_norm)):
            ops, trans = otf_ops_per_point(spins, kind)
            slots += n * (ops + TRANS_SLOTS * trans)
        sec = sh["mixed"]["stream_kernel_ms"] * 1e-3
        sh["roofline_mixed"] = {"bound": "alu", "achieved": slots / sec / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12,
                                "unit": "T lane-op slots/s", "frac": slots / sec / VALU_LANE_OPS_PEAK,
                                "slots_per_launch": slots, "kernel": f"k_eval<float,{synth.C4.n_res},true>",
                                "kernel_ms": sh["mixed"]["stream_kernel_ms"]}
        sh["fp64"]["mixed_speedup"] = sh["mixed"]["value"] / sh["fp64"]["value"]
        out["shapes_floated"] = sh
    if not args.no_small:
        out["smaller_workloads"] = smaller_workloads(args.steps, args.warmup)
    if not args.no_serve:
        out["serving"] = serving(args.serve_jobs, MIXED)
    if not args.no_paper_fit:
        out["paper_fit"] = paper_fit("fp64")
    if not args.no_cpu:
        cpu, vs = oracle_leg(wl, table, events, norm, mixed)
        log(f"[bench] oracle on the headline inputs: {cpu}; {vs}")
        vs["small_fit"] = small_fit_vs_oracle()
        log(f"[bench] small fit against the oracle's: {vs['small_fit']}")
        vs["headline_fit"] = headline_fit_mixed_vs_fp64(wl, table, events, norm)
        log(f"[bench] headline fit, mixed against FP64: {vs['headline_fit']}")
        out["vs_oracle"] = vs
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
