"""Shared test configuration.

Markers: ``gpu`` tests need an MI355X and call the HIP library through its C ABI; every other test
runs on the CPU (the oracle against its pins, host-side logic, the ABI's exported symbols).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU; runs the HIP library through its C ABI")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def gpu():
    """Skip-free gate: a gpu-marked test that runs without a GPU is an error, not a skip."""
    if not gpu_available():
        pytest.fail("gpu test selected but no GPU is visible")
    return True
