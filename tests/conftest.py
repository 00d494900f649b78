import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; skips the test when no GPU
    is visible (the binding itself raises if the library is missing)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2401_04865_amd import binding
    return binding
