import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu():
    """Skip unless a GPU is visible; with a GPU present the HIP library must load (no fallback)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2105_07372_amd import binding
    binding.load()           # raises if the extension is missing
    return torch.device("cuda:0")
