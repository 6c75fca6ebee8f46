import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def root():
    return ROOT


def oracle_model(workload, knots=None):
    """The oracle's model for a synthetic workload."""
    from oracle import Model, Res
    d = workload.decay
    kn = workload.knots() if knots is None else knots
    return Model(d.M, d.m1, d.m2, d.m3, d.rD, tuple(float(x) for x in kn),
                 tuple(Res(r.spin, r.mass, r.width, r.radius) for r in workload.resonances))


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(12345))
