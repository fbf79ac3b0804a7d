import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def mvp_ctx():
    """A libmvp context on cuda:0.  GPU tests fail (not skip) without a device
    or without the built library, so they can never pass on a fallback."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2103_01954_amd.api import Context
    ctx = Context(0)
    yield ctx
    import gc
    gc.collect()
    torch.cuda.synchronize()
