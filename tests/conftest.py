import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu():
    """Skips unless a GPU is present; fails loudly if the HIP library is missing there."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_09551_amd as msb
    msb.lib()                      # raises if libmsb.so is not built
    assert msb.msb_device_ok(), "device is not gfx950"
    return msb
