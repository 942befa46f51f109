import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library through its Python binding; fails loudly when absent."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test collected but no GPU is visible")
    from paper_1903_07884_amd import vie
    vie.load()
    return vie
