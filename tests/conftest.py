import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long statistical run")


_MELTS = {}


@pytest.fixture(scope="session")
def melt_c1():
    """The small parity melt: 16 chains x 16 beads, eta = 0.30, SAW with bond 1.2 sigma."""
    from paper_1502_06447_amd import inputs
    if "c1" not in _MELTS:
        _MELTS["c1"] = inputs.saw_chains(16, 16, 0.30, seed=1)
    return _MELTS["c1"]
