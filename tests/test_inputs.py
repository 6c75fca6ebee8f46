"""Seeded input recipes shared by the tests and the benchmark (no likelihood arithmetic here)."""
import numpy as np

import synth


def test_fit_start_holds_what_the_fit_holds():
    wl = synth.C1
    n_knots = 20
    truth = synth.truth_theta(n_knots, wl.resonances, 11)
    held = synth.fixed_mask(n_knots, wl.n_res).astype(bool)
    start = synth.fit_start(truth, n_knots, wl.n_res, 12)
    # the reference coefficient and the masses and widths keep their generated values
    assert np.array_equal(start[held], truth[held])
    assert held.sum() == 2 + 2 * wl.n_res
    # every floated parameter is moved, as perturb_theta moves it
    assert np.array_equal(start[~held], synth.perturb_theta(truth, n_knots, wl.n_res, 12)[~held])
    assert np.all(start[~held] != truth[~held])
    # seeded: the same seed gives the same start
    assert np.array_equal(start, synth.fit_start(truth, n_knots, wl.n_res, 12))
    # with the shapes floated only the reference coefficient is held
    floated = synth.fit_start(truth, n_knots, wl.n_res, 12, float_shapes=True)
    o = 2 * n_knots + 2 * wl.n_res
    assert np.all(floated[o:] != truth[o:])
