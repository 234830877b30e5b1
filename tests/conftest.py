import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP solver on cuda:0; GPU tests fail loudly without it."""
    import torch

    assert torch.cuda.is_available(), "GPU test collected without a GPU"
    from paper_2502_02460_amd import gevd

    gevd.load()
    return gevd
