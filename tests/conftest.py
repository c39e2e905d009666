import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library on cuda:0)")
    config.addinivalue_line("markers", "slow: long CPU work (full-size oracle runs)")


_RECORDS = []


@pytest.fixture
def record(request):
    """record(metric, value): keep a measured error for the parity report."""
    def add(metric, value):
        _RECORDS.append({"test": request.node.name, "metric": metric, "value": float(value)})
    return add


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("PARITY_REPORT")
    if path and _RECORDS:
        import json
        with open(path, "w") as f:
            json.dump(_RECORDS, f, indent=1)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle
