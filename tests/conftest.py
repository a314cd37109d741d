import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through libgfcc.so)")
    config.addinivalue_line("markers", "slow: long-running oracle test")
    import synth
    if not os.path.exists(synth._SO):
        synth.build()


@pytest.fixture(scope="session")
def gpu_ctx():
    import torch
    from paper_1902_06016_amd import gfcc
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = gfcc.Context(0)
    yield ctx
    ctx.close()
