import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and libhegrid.so")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Build the reference gridder once if it is not there yet."""
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
