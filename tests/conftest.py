import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library on a visible MI355X; GPU tests skip only when no GPU exists."""
    import ctypes
    import paper_1006_3340_amd as lll
    lib = lll.load()  # raises if the library is not built: no fallback path exists
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        n = ctypes.c_int(0)
        rc = hip.hipGetDeviceCount(ctypes.byref(n))
    except OSError:
        rc, n = 1, ctypes.c_int(0)
    if rc != 0 or n.value < 1:
        pytest.skip("no HIP device visible")
    return lll
