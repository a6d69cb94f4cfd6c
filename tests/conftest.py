import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


@pytest.fixture(scope="session")
def hb():
    """The HIP library binding; fails loudly when there is no GPU."""
    import paper_2604_08374_amd as hb

    n = hb.device_count()
    if n < 1:
        pytest.fail("no GPU visible: the GPU tests run the HIP library and have no fallback")
    return hb
