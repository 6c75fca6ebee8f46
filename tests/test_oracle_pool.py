"""The oracle split over worker processes gives the oracle's own results (CPU)."""
import numpy as np

import synth
from oracle import kinematics as K
from oracle import likelihood as L
from oracle.pool import OraclePool
from tests.conftest import oracle_model


def test_pool_equals_the_single_process_oracle():
    wl = synth.C4
    m = oracle_model(wl)
    ev = synth.uniform_phase_space(wl.decay, 7000, 71)
    n12, n13 = synth.uniform_phase_space(wl.decay, 9000, 72)
    w = np.full(len(n12), K.area(m) / len(n12))
    eps = 0.5 + 0.5 * np.cos(n12) ** 2
    th = wl.start()
    with OraclePool(m, ev, (n12, n13, w * eps), log_eps_sum=1.25, w_plain=w, workers=2, chunk=2500) as pool:
        for shapes in (False, True):
            v, g = pool.nll_and_grad(th, shapes=shapes)
            v_o, g_o = L.nll_and_grad(m, th, ev, (n12, n13, w * eps), 1.25, shapes=shapes)
            assert abs(v - v_o) <= 1e-12 * abs(v_o)
            assert np.abs(g - g_o).max() <= 1e-10 * np.abs(g_o).max()
        I = pool.integrals(th)
        I_o = L.integrals(m, th, (n12, n13, w))
        assert np.abs(I - I_o).max() <= 1e-12 * np.abs(I_o).max()
        free = np.flatnonzero(wl.fixed() == 0)
        sig = pool.expected_sigma(th, free, 4000)
        assert np.all(sig[free] > 0) and np.all(sig[wl.fixed() == 1] == 0)
