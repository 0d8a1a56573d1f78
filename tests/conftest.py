import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


@pytest.fixture(scope="session")
def c3_full():
    """The 4,000,000-atom jittered FCC system of the benchmark and its oracle
    neighbour sets (built once per session)."""
    import workloads as W
    from helpers import oracle_neighbors
    w = W.c3()
    sy = w.systems[0]
    row, col = oracle_neighbors(sy, w.r_cut)
    return w, sy, row, col
