import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


@pytest.fixture(autouse=True)
def _progress_to_terminal(request, capsys):
    """GPU tests print the case they are about to run through gpu_cases.say; route
    those lines past pytest's capture so that they appear while the test runs."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    import gpu_cases

    def sink(msg):
        with capsys.disabled():
            print(msg, flush=True)

    gpu_cases._sink = sink
    try:
        yield
    finally:
        gpu_cases._sink = None
