import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")
    config.addinivalue_line("markers", "blas_threads: the oracle work of this test is large enough "
                                       "(benzene-sized) to use every BLAS thread")


@pytest.fixture(autouse=True)
def _blas_threads(request):
    """The oracle's small factorisations and products (c1 and smaller) run many
    times faster on one BLAS thread than on a many-core pool, whose start-up
    cost per call dominates at these sizes; tests marked blas_threads keep the
    whole pool."""
    if request.node.get_closest_marker("blas_threads"):
        yield
        return
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        yield
        return
    with threadpool_limits(limits=1, user_api="blas"):
        yield
