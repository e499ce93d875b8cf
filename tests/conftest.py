"""Shared test setup: the `gpu` marker and import paths.

Tests marked `gpu` need an MI355X and the built HIP library; everything else
runs on the CPU (the oracle pins, host logic, the C-ABI symbol check).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    return O


@pytest.fixture(scope="session")
def oracle3_mod():
    from oracle import oracle as O
    from oracle import oracle3 as O3
    if not os.path.exists(O.LIB3):
        O.build()
    return O3
