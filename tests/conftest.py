import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: long-running check (still part of the default suite)")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build(force=False)
    yield


@pytest.fixture(scope="session", autouse=True)
def _library_built():
    """Load the built HIP library; build it only if nothing is built yet."""
    import paper_2310_00236_amd as hw
    if not os.path.exists(hw.LIB_PATH):
        from paper_2310_00236_amd import build
        build.build()
    yield
