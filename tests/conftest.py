import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.load()
    return oracle


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session", autouse=True)
def _hip_library_built():
    """Build libamg355.so in-tree when it is absent (a fresh checkout); an
    existing build is used as it is."""
    from paper_2606_09001_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2606_09001_amd.csrc import build
        build.build()
