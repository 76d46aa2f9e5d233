import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def _stale(lib, srcdir, exts):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    for f in os.listdir(srcdir):
        if f.endswith(exts) and os.path.getmtime(os.path.join(srcdir, f)) > t:
            return True
    return False


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if _stale(oracle.LIB, oracle.HERE, (".cpp", ".hpp")):
        oracle.build()
    yield
