import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only test")


def pytest_sessionstart(session):
    # the oracle's worker processes fork from a clean server process started
    # here, before any test touches the GPU
    from oracle import pool
    pool.start()
