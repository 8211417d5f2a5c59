import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on the GPU)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(autouse=True)
def _announce_gpu_test(request):
    # Name the case before any GPU work so a crash can be traced to it.
    if request.node.get_closest_marker("gpu") is not None:
        sys.stderr.write(f"\n[gpu-test] {request.node.nodeid}\n")
        sys.stderr.flush()
    yield
