import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-side check")


@pytest.fixture(scope="session", autouse=True)
def _oracle_lib():
    """The plain-C oracle is rebuilt when its source is newer than the library."""
    from oracle import clib
    clib.build(force=False)
    yield
