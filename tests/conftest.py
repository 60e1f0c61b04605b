import os
import sys

import pytest

# The serve loop overlaps requests on separate streams; HIP maps a process's
# streams round-robin onto GPU_MAX_HW_QUEUES hardware queues (4 by default),
# and two streams on one queue run one after the other.  Set before any HIP
# initialisation in this process.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")
