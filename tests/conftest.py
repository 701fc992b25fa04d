import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def ctx():
    """One lsr context on cuda:0, ordered against torch's current stream."""
    import torch

    import paper_1609_04567_amd as L
    assert torch.cuda.is_available(), "GPU tests need a device"
    c = L.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()
