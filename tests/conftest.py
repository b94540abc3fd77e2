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


# Batches of the posterior-moment comparisons.  A batch-means standard error
# is only right when each batch spans many autocorrelation times; the theta
# chains here have integrated autocorrelation times of 140-220 cycles (BB1,
# N = 400), so floor(sqrt(M)) batches of ~155 draws out of M = 24,000 would
# understate the error ~1.8-fold, while 30 batches of 800 draws do not.
MOMENT_BATCHES = 30

# Key of the oracle chains that free-run moment tests compare with a GPU
# chain: a different Philox key from the workload's, so that the two chains
# are independent (with the same key they would agree draw for draw until
# rounding first flips a decision, and the combined standard error of their
# difference would be too large).
INDEPENDENT_SEED = 1000003


def moment_scores(a: np.ndarray, b: np.ndarray, n_batches: int = MOMENT_BATCHES):
    """Per component of two chains [M][p]: the difference of their means and
    of their variances in units of the combined batch-means standard error,
    |m_a - m_b| / sqrt(se_a^2 + se_b^2), as (z_mean, z_var, m_a, se_a, m_b, se_b)."""
    out = []
    for j in range(a.shape[1]):
        ma, sa = batch_means(a[:, j], n_batches)
        mb, sb = batch_means(b[:, j], n_batches)
        va, sva = batch_means((a[:, j] - ma) ** 2, n_batches)
        vb, svb = batch_means((b[:, j] - mb) ** 2, n_batches)
        out.append((abs(ma - mb) / np.hypot(sa, sb), abs(va - vb) / np.hypot(sva, svb), ma, sa, mb, sb))
    return out


def assert_moments_agree(scores, rms_bound: float = 2.0, each_bound: float = 4.0):
    """Posterior means and variances within 2 combined standard errors, pooled
    over the 2p moments: the root mean square of their z-scores below 2 (under
    agreement the sum of squares is about chi-square with 2p degrees of
    freedom: a false alarm has probability about 0.3 % at p = 2 and below
    0.1 % for p >= 3), and no single moment beyond 4 (with 29 degrees of
    freedom in each standard error, 0.4 % over ten moments)."""
    z = np.array([[s[0], s[1]] for s in scores]).ravel()
    rms = float(np.sqrt(np.mean(z ** 2)))
    assert rms < rms_bound and z.max() < each_bound, (rms, z.tolist())
    return rms
