import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session", autouse=True)
def _release_library_objects():
    """Destroy every libpm object at the end of the session, while the HIP
    runtime is fully alive, whatever tracebacks still reference them."""
    yield
    import sys
    pm = sys.modules.get("paper_1808_10580_amd")
    if pm is not None:
        pm.release_all()
