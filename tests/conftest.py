import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def c1_graph():
    from synth import config_graph
    g, _, _, _ = config_graph("C1")
    return g


@pytest.fixture(scope="session")
def c1_tables(c1_graph):
    import oracle
    g = c1_graph
    return oracle.Tables(g.n, g.src, g.dst, g.w)
