import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU oracle run (still part of the CPU suite)")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built product library; a GPU test fails loudly if it is missing."""
    from paper_2107_06355_amd import lbm

    lbm.load()
    return lbm
