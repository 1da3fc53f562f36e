import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(scope="session")
def dgf64_q4():
    from oracle.dgf import dgf_cached
    return dgf_cached(4, 64)


@pytest.fixture(scope="session")
def dgf64_q6():
    from oracle.dgf import dgf_cached
    return dgf_cached(6, 64)
