import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs through the C-ABI library")
    config.addinivalue_line("markers", "slow: a longer CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def mdfs_gpu():
    """The C-ABI binding on cuda:0.  Skips only when no GPU is present; a missing library on a
    GPU machine is an error, not a skip."""
    if not gpu_available():
        pytest.skip("no GPU in this environment")
    from paper_1811_00631_amd import mdfs
    mdfs.load()  # raises if the HIP library is missing
    return mdfs
