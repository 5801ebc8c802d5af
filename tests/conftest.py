import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


def pytest_sessionfinish(session, exitstatus):
    """With SBS_PARITY_LOG set, write the FP32 cost errors the parity checks
    observed (one record per check) to that file as JSON."""
    path = os.environ.get("SBS_PARITY_LOG")
    if not path:
        return
    try:
        import parity_util
    except ImportError:
        return
    import json
    with open(path, "w") as f:
        json.dump([{"test": t, "max_rel": a, "max_abs": b, "median_rel": m, "samples": n}
                   for t, a, b, m, n in parity_util.OBSERVED], f, indent=1)
