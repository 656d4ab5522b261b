import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Build the C oracle once if it is not there yet (gcc, a second)."""
    lib = os.path.join(ROOT, "oracle", "liborc_direct.so")
    if not os.path.exists(lib):
        from oracle.build import build
        build()
    yield
