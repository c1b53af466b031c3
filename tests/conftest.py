import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """Skip-free guard: a test marked gpu fails loudly when no GPU or no library is present."""
    if not _gpu_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2208_10839_amd import binding
    binding.load()  # raises if the HIP library is missing
    return binding
