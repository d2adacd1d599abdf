import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def sphere3k():
    import synth
    return synth.unit_sphere(3000)


@pytest.fixture(scope="session")
def sphere3k_dense(sphere3k):
    from oracle import dense
    s = sphere3k
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    return a, dense.DenseLU(a)


@pytest.fixture(scope="session")
def sphere3k_rss(sphere3k):
    from oracle import rss
    s = sphere3k
    return rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps,
                         check_invariant=True, brute_force_check=True)
