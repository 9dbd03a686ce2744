import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def c1_problem():
    """c1 inputs and the oracle's projected Hamiltonian (CSR)."""
    import synth
    from oracle import hamiltonian, space
    w = synth.WORKLOADS["c1"]
    h, g = w.integrals()
    keys = space.full_space(w.n, w.na, w.nb)
    Hm = hamiltonian.build(keys, w.n, h, g)
    return dict(w=w, h=h, g=g, keys=keys, H=Hm, theta=w.theta())
