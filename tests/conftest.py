import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _keep_large_allocations_on_the_heap():
    """glibc serves large blocks (NumPy's temporaries of the oracle, tens of MB) by mmap and unmaps
    them when freed, so every fresh temporary page-faults in again; on the virtual machines the tests
    run on that dominates the oracle's time.  Raising the mmap and trim thresholds keeps freed blocks
    for reuse (M_MMAP_THRESHOLD = -3, M_TRIM_THRESHOLD = -1 in malloc.h).  Arithmetic is unchanged."""
    try:
        import ctypes
        libc = ctypes.CDLL("libc.so.6")
        libc.mallopt(-3, 1 << 30)
        libc.mallopt(-1, 1 << 31)
    except (OSError, AttributeError):
        pass


_keep_large_allocations_on_the_heap()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def wl0():
    import synth
    return synth.make_workload("cfg0")


@pytest.fixture(scope="session")
def wl1():
    import synth
    return synth.make_workload("cfg1")


@pytest.fixture(scope="session")
def wl2():
    import synth
    return synth.make_workload("cfg2")
