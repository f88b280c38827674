import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def okeys():
    """Oracle keys at the default parameters (seed 1), shared by the session."""
    import oracle
    return oracle.keygen(1)


@pytest.fixture(scope="session")
def octx(okeys):
    import oracle
    return oracle.Ctx(okeys)
