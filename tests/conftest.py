import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle


@pytest.fixture(autouse=True)
def _gpu_memory_release(request):
    """After every GPU test: free the library's cached work buffers and torch's cache, so
    that large tests do not starve the next ones of device memory."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    import torch
    if not torch.cuda.is_available():
        return
    from paper_2201_09729_amd import dlma
    torch.cuda.synchronize()
    dlma.dlma_release_cache()
    torch.cuda.empty_cache()
