import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """The oracle and the workload generator are host C; build them if absent."""
    import oracle
    import workloads
    if not os.path.exists(oracle._SO):
        oracle.build()
    if not os.path.exists(workloads._SO):
        workloads.build()
    yield
