import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through its C ABI)")
    config.addinivalue_line("markers", "slow: long-running statistical or full-size case")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this container")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()


@pytest.fixture(autouse=True)
def _progress_log(request):
    """With ISING_PROGRESS_LOG set, append each test id (flushed) before it runs,
    so a run that dies on the GPU still names the case it was in."""
    path = os.environ.get("ISING_PROGRESS_LOG")
    if path:
        import time
        with open(path, "a") as f:
            f.write(f"{time.strftime('%H:%M:%S')} START {request.node.nodeid}\n")
            f.flush()
    yield
