import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Compile the CPU oracle once per session (test infrastructure)."""
    from oracle import oracle as O
    libs = (O.LIB_PATH, O.LIB_PATH_EXT)
    if any(not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(O.SRC_PATH)
           for p in libs):
        O.build()
    yield
