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
        return bool(torch.cuda.is_available())
    except Exception:
        return False


@pytest.fixture(scope="session")
def gr():
    """The HIP library binding; fails loudly if it is not built or no GPU."""
    if not gpu_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    import paper_2602_01057_amd as pkg
    pkg.load_library()
    return pkg
