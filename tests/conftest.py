import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


import pytest


@pytest.fixture(scope="session")
def lib_or_skip():
    """The ctypes handle of libcwth.so (built on demand); host-only entry
    points can be called without a device."""
    from paper_2408_14302_amd import build
    lib_path = os.path.join(ROOT, "paper_2408_14302_amd", "libcwth.so")
    if not os.path.exists(lib_path):
        build.build(verbose=False)
    from paper_2408_14302_amd import cwth
    return cwth.raw()
