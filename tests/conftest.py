import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def batch_means(x: np.ndarray, n_batches: int = None):
    """Mean and batch-means Monte Carlo standard error along axis 0."""
    x = np.asarray(x, dtype=np.float64)
    m = x.shape[0]
    b = n_batches or max(2, int(np.floor(np.sqrt(m))))
    size = m // b
    xb = x[: b * size].reshape(b, size, *x.shape[1:]).mean(axis=1)
    return x[: b * size].mean(axis=0), xb.std(axis=0, ddof=1) / np.sqrt(b)
