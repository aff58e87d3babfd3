"""Shared fixtures.  Tests marked ``gpu`` need an MI355X; everything else runs
on the CPU (oracle pins, host logic, library loading)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU (runs the HIP kernels through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import build_oracle
    from oracle import oracle as O

    if not os.path.exists(O.LIB_PATH):
        build_oracle.build()
    return O.load()


@pytest.fixture(scope="session")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19941_amd import dsm

    dsm.load()  # raises if the HIP library is missing: there is no fallback
    return torch.device("cuda:0")


def f32(a):
    """Round to float32 and back: inputs both implementations see identically."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)
