import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="session")
def nthreads():
    return _threads()


@pytest.fixture(scope="session")
def tiny_build():
    """(workload, index, db, queries) for a small GMM workload, built by the oracle."""
    import datagen
    import oracle
    w = datagen.small()
    ix, db, q = oracle.build_workload(w, nthreads=_threads())
    return w, ix, db, q


@pytest.fixture(scope="session")
def c1_build():
    """(workload, index, db, queries) for the 10k-vector workload, built by the oracle."""
    import datagen
    import oracle
    w = datagen.C1
    ix, db, q = oracle.build_workload(w, nthreads=_threads())
    return w, ix, db, q
