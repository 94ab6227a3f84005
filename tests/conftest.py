import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def pytest_sessionstart(session):
    """Native stack traces for crashes in the test process (after faulthandler is set up,
    so its Python traceback still follows)."""
    import ctypes
    lib = os.path.join(ROOT, "tests", "libnative_backtrace.so")
    if os.path.exists(lib):
        ctypes.CDLL(lib).native_backtrace_install()
