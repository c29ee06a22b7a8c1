import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: a longer CPU or GPU case")


def _step(msg):
    print(msg, flush=True)


@pytest.fixture(autouse=True)
def _announce(request):
    # names the case before any GPU work, so a run that dies mid-test still says which
    if request.node.get_closest_marker("gpu") is not None:
        _step(f"\n[gpu-case] {request.node.nodeid}")
    yield
