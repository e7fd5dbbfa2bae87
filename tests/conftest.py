import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Pin the system HIP runtime before anything imports torch (see the package docstring).
import paper_2301_05451_amd  # noqa: E402,F401


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libtq.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")
