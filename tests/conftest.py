"""Shared test configuration.

Tests marked ``gpu`` need an MI355X and the built HIP library; everything
else runs on the CPU and checks the oracle against what the paper and the
mathematics fix."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built libsfmm.so")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
