import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(autouse=True)
def _no_device_errors(request):
    """Every GPU test ends with the device's error word clear: a table bound
    exceeded anywhere in the library fails the test that caused it."""
    yield
    if "gpu" not in request.keywords or not _gpu_available():
        return
    from paper_1410_6754_amd import api
    bits = api.device_errors(clear=True)
    assert bits == 0, "device error bits 0x%x raised during the test" % bits
