import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

try:  # the oracle's many tiny factorizations run fastest single-threaded
    import numpy  # noqa: F401  -- the BLAS must be loaded before its threads are limited
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
except Exception:  # pragma: no cover
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
