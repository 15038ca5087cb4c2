import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libnb.so")
    config.addinivalue_line("markers", "slow: long CPU test")


def _ensure_libnb():
    from paper_1506_00716_amd import nb
    if not os.path.exists(nb.LIB_PATH):
        from paper_1506_00716_amd import build
        build.build()
    return nb


@pytest.fixture(scope="session")
def nbmod():
    """The libnb binding module (library built in-tree if missing)."""
    return _ensure_libnb()


@pytest.fixture(scope="session")
def gpu_ctx(nbmod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return nbmod.Context(0)
