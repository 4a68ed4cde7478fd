import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True)
def _gpu_progress(request):
    """Records each GPU test before it runs, in FPS_TEST_PROGRESS_DIR (if set),
    flushed to disk: after a crash the last line names the case."""
    d = os.environ.get("FPS_TEST_PROGRESS_DIR")
    if d and request.node.get_closest_marker("gpu") is not None:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "gpu_test_progress.log"), "a") as f:
            f.write(f"START {request.node.nodeid}\n")
            f.flush()
            os.fsync(f.fileno())
    yield
