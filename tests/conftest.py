"""Shared test configuration.

Markers:
  gpu  -- needs an MI355X (runs the GPU library through its C ABI).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: test needs an AMD Instinct GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        O.build()
    return O
