import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the GPU)")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


@pytest.fixture(scope="session")
def cube5():
    from gen import make_problem
    return make_problem(5)


@pytest.fixture(scope="session", autouse=True)
def _close_library_objects():
    """Close every Hierarchy / EdgeNet a test left open when the session ends (before the
    interpreter shuts down), instead of leaving them to garbage collection at exit."""
    yield
    import paper_2011_13325_amd as E
    E.close_all()
