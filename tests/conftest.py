import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


LIB = os.path.join(ROOT, "paper_1001_1588_amd", "libfftenkf.so")


@pytest.fixture(scope="session")
def built_lib():
    """Path of libfftenkf.so, built in-tree first if nothing is built yet."""
    if not os.path.exists(LIB):
        from paper_1001_1588_amd import build
        build.build()
    return LIB
