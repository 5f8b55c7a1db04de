import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_parts():
    """The generator and the oracle are plain C: build them if missing."""
    import oracle
    import qm_inputs
    if not os.path.exists(qm_inputs._SO):
        qm_inputs.build()
    if not os.path.exists(oracle._SO):
        oracle.build()
    yield
