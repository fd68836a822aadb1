import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP library")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """Build the two host-only helper libraries (gcc, seconds) once per session."""
    import oracle
    import workloads
    for mod, src in ((oracle, oracle._SRC), (workloads, workloads._SRC)):
        stale = not os.path.exists(mod._LIB) or os.path.getmtime(mod._LIB) < os.path.getmtime(src)
        mod.build(force=stale)
    yield
