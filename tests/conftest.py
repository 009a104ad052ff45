import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True)
def _fresh_tuning():
    """Every test starts from the default launch shapes: the autotuner's per-process
    choices (recorded by an earlier test) are forgotten before each test."""
    try:
        from paper_1008_0502_amd import _lib
        if _lib._LIB is not None:
            _lib._LIB.sp_tune_cache_clear()
    except Exception:
        pass
    yield
