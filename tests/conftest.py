import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _ensure_cpu_libs():
    # The generator and the oracle are plain gcc builds; build them if absent
    # so that the CPU suite runs from a clean checkout.
    import lpgen
    import oracle
    if not os.path.exists(lpgen.LIB_PATH):
        lpgen.build()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def olib():
    import oracle
    return oracle.lib()
