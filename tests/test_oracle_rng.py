"""Pins for the oracle's random numbers.

The counter-based generator is Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
SC'11); the paper only names the CUDA random-number library it used
(Sec. 2.2), so the stream layout is this project's own: key = seed,
counter = (object, sweep, tag, block).  Pins:
  * rocRAND's independent Philox4x32-10 implementation, compiled from its
    public header and run on the host, must give the same 128-bit blocks;
  * the 24-bit field cut and the (field + 1) 2^-24 map are checked bit by
    bit with Python integers;
  * Box-Muller output must be standard normal (moments, KS test).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_bin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers or hipcc not available")
    out = str(tmp_path_factory.mktemp("rr") / "rocrand_philox")
    subprocess.run([hipcc, "-O1", "-o", out, os.path.join(HERE, "pins", "rocrand_philox.cpp")],
                   check=True, capture_output=True)
    return out


def _cases():
    rng = np.random.default_rng(42)
    cases = [(0, 0, 0, 0, 0), (2**64 - 1, 0, 0, 0, 0), (0, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1),
             (1, 999_999, 5000, 0, 0), (1000, 0, 17, 1, 3), (1000, 0, 17, 2, 0)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                      int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
                      int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))))
    return cases


def test_philox_matches_rocrand(oracle_lib, rocrand_bin):
    cases = _cases()
    inp = "".join(f"{s} {a} {b} {c} {d}\n" for s, a, b, c, d in cases)
    res = subprocess.run([rocrand_bin], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in ln.split()] for ln in res.stdout.strip().splitlines()], dtype=np.uint64)
    assert ref.shape == (len(cases), 4)
    for (s, a, b, c, d), r in zip(cases, ref):
        key = [s & 0xFFFFFFFF, s >> 32]
        got = oracle_lib.philox4x32_10([a, b, c, d], key)
        assert list(got.astype(np.uint64)) == list(r), (s, a, b, c, d)


def test_field_cut_and_uniform_map(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(300):
        seed = int(rng.integers(0, 2**63))
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        x = oracle_lib.philox4x32_10(ctr, [seed & 0xFFFFFFFF, seed >> 32])
        v = int(x[0]) | (int(x[1]) << 32) | (int(x[2]) << 64) | (int(x[3]) << 96)
        u, z = oracle_lib.variates(seed, ctr)
        for j in range(5):
            field = (v >> (24 * j)) & 0xFFFFFF
            # exact: u * 2^24 is the integer field + 1, so u lies in (0, 1]
            assert u[j] * 16777216.0 == field + 1
        r0 = np.sqrt(-2.0 * np.log(u[0]))
        assert z[0] == pytest.approx(r0 * np.cos(2 * np.pi * u[1]), rel=1e-14, abs=1e-14)
        assert z[3] == pytest.approx(np.sqrt(-2.0 * np.log(u[2])) * np.sin(2 * np.pi * u[3]), rel=1e-14, abs=1e-14)


def test_variates_are_uniform_and_normal(oracle_lib):
    n = 40000
    us = np.zeros((n, 5))
    zs = np.zeros((n, 4))
    for i in range(n):
        us[i], zs[i] = oracle_lib.variates(3, [i, 11, 0, 0])
    for j in range(5):
        assert stats.kstest(us[:, j], "uniform").pvalue > 1e-4
    for j in range(4):
        assert stats.kstest(zs[:, j], "norm").pvalue > 1e-4
        assert abs(zs[:, j].mean()) < 5.0 / np.sqrt(n)
        assert abs(zs[:, j].var() - 1.0) < 6.0 * np.sqrt(2.0 / n)
    # the two normals of one Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(zs[:, 0], zs[:, 1])[0, 1]) < 5.0 / np.sqrt(n)


def test_streams_differ_by_key_and_tag(oracle_lib):
    a = oracle_lib.philox4x32_10([5, 9, 0, 0], [1, 0])
    b = oracle_lib.philox4x32_10([5, 9, 0, 0], [2, 0])
    c = oracle_lib.philox4x32_10([5, 9, 1, 0], [1, 0])
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
