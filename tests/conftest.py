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
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")


def pytest_sessionstart(session):
    """Build the library once if it is missing (hipcc cross-compiles without a GPU)."""
    lib = os.path.join(ROOT, "paper_2503_21206_amd", "libpilotann.so")
    if not os.path.exists(lib):
        from paper_2503_21206_amd.build import build
        build()
