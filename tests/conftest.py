import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The loaded C-ABI library on a machine with a GPU; fails loudly when it is
    missing."""
    from paper_2608_03894_amd import kdqmc
    lib = kdqmc.load()
    if not kdqmc.gpu_available():
        pytest.fail("no GPU visible to HIP")
    return lib
