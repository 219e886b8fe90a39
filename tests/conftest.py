"""Shared pytest configuration: the ``gpu`` marker and GPU availability helpers."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def gpu_ok():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    return True


@pytest.fixture(scope="session")
def semlib():
    """The ctypes binding; builds the library first if it is not built yet."""
    lib = os.path.join(ROOT, "paper_2104_08416_amd", "libsem_hip.so")
    if not os.path.exists(lib):
        from paper_2104_08416_amd import build
        build.build()
    from paper_2104_08416_amd import sem
    return sem
