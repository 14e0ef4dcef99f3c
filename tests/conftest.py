"""Test configuration: the `gpu` marker and shared helpers.

CPU tests (``-m "not gpu"``) pin the oracle against closed forms, the paper's printed
values and brute force, check the input generators and the host side of the C ABI.
GPU tests (``-m gpu``) compare the HIP path, called through the C ABI, with the oracle.
"""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")


@pytest.fixture(scope="session")
def oracle():
    import oracle as o
    o.build()
    return o


def interior(dim):
    return (slice(1, -1),) * dim


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
