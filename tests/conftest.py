import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Several test processes at once (pytest-xdist workers): the oracle's OpenMP threads of
# every worker share the cores, and spin-waiting threads then starve each other; they
# wait passively instead (read when the oracle library first loads, after this module).
if os.environ.get("PYTEST_XDIST_WORKER"):
    os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")
