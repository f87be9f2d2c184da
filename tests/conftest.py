import os
import sys

import pytest

# HIP maps streams onto a per-process pool of hardware queues (4 by default); past that,
# streams share queues and their work runs one after another. The GPU tests create a few
# streams per test (the serving slots' own get queues outside the pool): eight queues keep
# them apart. Set before the HIP runtime starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
