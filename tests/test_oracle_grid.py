"""The evenly spaced normalisation grid of Sec. 4 (spacings of Fig. 2) and the normalisation integral
computed on it.

Pins: the number of grid points times the cell area against the region's area by quadrature, within
the bound set by the cells the boundary crosses; the grid integral of |A|^2 against an independent
Monte Carlo estimate; and its convergence as the spacing shrinks, which is the effect Fig. 2 shows.
"""
import math

import numpy as np
import pytest

import synth
from oracle import kinematics as K
from oracle import likelihood as L
from tests.conftest import oracle_model

SPACINGS = (0.01, 0.004, 0.001)


@pytest.mark.parametrize("wl", [synth.C1, synth.KKK], ids=["pipipi", "kkk"])
def test_grid_count_times_cell_area_is_the_area(wl):
    d = wl.decay
    area = K.area(oracle_model(wl))
    # The region is convex, so its boundary is no longer than the perimeter of the bounding square;
    # only cells the boundary crosses can be miscounted, at most sqrt(2) L / spacing + 4 of them.
    perimeter = 4.0 * (d.smax - d.smin)
    errs = []
    for h in SPACINGS:
        s12, s13, w = synth.grid_points(d, h)
        assert np.all(w == h * h)
        assert np.all(synth.inside_region(d, s12, s13))
        err = abs(len(s12) * h * h - area)
        assert err <= math.sqrt(2.0) * perimeter * h + 4.0 * h * h, (h, err)
        errs.append(err / area)
    assert errs[-1] < 1e-4


def test_grid_points_are_cell_centres_on_the_anchored_lattice():
    d = synth.C1.decay
    h = 0.01
    s12, s13, _ = synth.grid_points(d, h)
    for s in (s12, s13):
        k = (s - d.smin) / h - 0.5
        assert np.allclose(k, np.round(k), atol=1e-9)
    # every lattice centre inside the region is present, none twice
    i = np.floor((s12 - d.smin) / h).astype(int)
    j = np.floor((s13 - d.smin) / h).astype(int)
    assert len(set(zip(i, j))) == len(s12)
    # and a centre the grid left out is outside the region
    lat = d.smin + (np.arange(int(math.ceil((d.smax - d.smin) / h))) + 0.5) * h
    X, Y = np.meshgrid(lat, lat, indexing="ij")
    assert int(synth.inside_region(d, X, Y).sum()) == len(s12)


def test_grid_normalisation_converges_to_the_monte_carlo_integral():
    """K-K+K+ at the truth: the phi(1020) peak (m Gamma ~ 0.004 GeV^2 wide in s) makes the coarse grids
    visibly wrong; the 0.001 grid agrees with a 4M-point Monte Carlo estimate within its error."""
    wl = synth.KKK
    m = oracle_model(wl)
    th = wl.truth()
    vals = {}
    for h in SPACINGS:
        vals[h] = L.norm_integral(m, th, synth.grid_points(wl.decay, h))
    n = 4_000_000
    s12, s13 = synth.uniform_phase_space(wl.decay, n, 77)
    area = K.area(m)
    a = L.amplitude(m, th, s12, s13)
    f = a.real ** 2 + a.imag ** 2
    mc, err = area * f.mean(), area * f.std() / math.sqrt(n)
    d01, d004, d001 = (abs(vals[h] - mc) for h in SPACINGS)
    assert d001 <= 4.0 * err, (vals, mc, err)
    assert abs(vals[0.004] - vals[0.001]) < abs(vals[0.01] - vals[0.001])
