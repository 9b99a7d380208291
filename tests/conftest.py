import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def pytest_sessionstart(session):
    """Load what is built; build the HIP library only when none exists."""
    from paper_2510_13310_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2510_13310_amd.build import build
        build()
