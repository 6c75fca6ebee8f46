"""mipwa_eval_noalloc through the C ABI: the same results as mipwa_eval_async, with its scratch in the
library's static per-GPU array.  Two calls in a row, the second on a smaller input; each context's
first evaluation is the no-alloc one (nothing of the context's own launch state exists yet)."""
import ctypes as C

import numpy as np
import pytest

import synth
from tests.cases import make_problem, rel

pytestmark = pytest.mark.gpu


def _call(ctx, name, theta):
    import torch
    ctx.set_params(theta)
    out = torch.full((1 + ctx.n_params,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    rc = getattr(ctx._lib, name)(ctx._h, C.c_void_p(st.cuda_stream), C.c_void_p(out.data_ptr()))
    assert rc == 0, (name, rc, ctx._lib.mipwa_last_error(ctx._h).decode())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_equals_async_calls_in_a_row_each_smaller():
    """Three contexts in a row, each smaller than the one before: 50 knots and three resonances in
    FP64 (its tables go up through device memory), then 40 knots in mixed precision, then 20 knots in
    FP64 (tables in the kernel arguments)."""
    from paper_1703_03284_amd import FP64, MIXED
    for wl, n_ev, n_nm, prec in ((synth.C4, 100_000, 300_000, "fp64"), (synth.C2, 50_000, 150_000, "mixed"),
                                 (synth.C1, 3000, 20000, "fp64")):
        print(f"noalloc case: {wl.name} {n_ev}+{n_nm} {prec}", flush=True)
        prob = make_problem(wl, n_ev, n_nm, seed=61 + n_ev % 7)
        ctx = prob.context(MIXED if prec == "mixed" else FP64)
        th = prob.theta.copy()
        th2 = th.copy()
        th2[-3] += 0.003   # a mass: the resonance cache is rebuilt by the no-alloc call
        th2[0] *= 1.02
        got = [_call(ctx, "mipwa_eval_noalloc", t) for t in (th, th2, th)]
        ref = [_call(ctx, "mipwa_eval_async", t) for t in (th, th2, th)]
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (np.abs(g - r).max())
        # and to the oracle at the parity bar of the precision
        v_o, g_o = prob.oracle(theta=th2)
        n_ck = 2 * wl.n_knots + 2 * wl.n_res
        tol_v, tol_g = (1e-10, 1e-8) if prec == "fp64" else (1e-6, 1e-4)
        assert rel(got[1][0], v_o) <= tol_v
        assert np.abs(got[1][1:1 + n_ck] - g_o[:n_ck]).max() <= tol_g * np.abs(g_o[:n_ck]).max()
        ctx.close()


def test_noalloc_rejects_what_it_cannot_hold():
    import torch
    from paper_1703_03284_amd import FP64, NORM_QFORM
    big = synth.Workload("max_model", 9, "fp64", 20000, 20000, 128,
                         (synth.RHO770, synth.F2_1270, synth.RHO1450, synth.F0_980), "flat", float_shapes=True)
    prob = make_problem(big, big.n_events, big.n_norm, seed=63)
    ctx = prob.context(FP64)
    ctx.set_fixed(big.fixed())
    ctx.set_launch(blocks=4096, waves=1)   # 4096 blocks x 1041-double records: beyond the 8 MiB array
    out = torch.zeros(1 + ctx.n_params, dtype=torch.float64, device="cuda")
    rc = ctx._lib.mipwa_eval_noalloc(ctx._h, None, C.c_void_p(out.data_ptr()))
    assert rc == -1
    assert "scratch" in ctx._lib.mipwa_last_error(ctx._h).decode()
    ctx.close()
    small = make_problem(synth.C1, 2000, 10000, seed=64)
    ctx = small.context(FP64)
    ctx.set_norm_mode(NORM_QFORM)
    out = torch.zeros(1 + ctx.n_params, dtype=torch.float64, device="cuda")
    assert ctx._lib.mipwa_eval_noalloc(ctx._h, None, C.c_void_p(out.data_ptr())) == -4
    ctx.close()
