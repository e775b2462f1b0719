import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def xyl():
    """The HIP product binding; fails loudly (never falls back) when it cannot load."""
    if not gpu_available():
        pytest.fail("GPU test selected but no GPU is visible")
    import paper_2409_06412_amd as xyl_mod
    xyl_mod.load()
    return xyl_mod
