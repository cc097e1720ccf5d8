import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


_PROGRESS = os.environ.get("FDC_TEST_PROGRESS_DIR")
_count = [0]


@pytest.fixture(autouse=True)
def _progress_marker(request):
    """With FDC_TEST_PROGRESS_DIR set, write one small file per finished test
    (name and wall time), so a long test run shows its progress as it goes."""
    import time
    t0 = time.time()
    yield
    if _PROGRESS:
        _count[0] += 1
        os.makedirs(_PROGRESS, exist_ok=True)
        with open(os.path.join(_PROGRESS, f"test_{_count[0]:03d}.txt"), "w") as f:
            f.write(f"{request.node.nodeid} {time.time() - t0:.2f}s\n")
