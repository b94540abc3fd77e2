"""Pins for the oracle's selection normaliser Z(theta) (eq 4.4 denominator).

Z(theta) = int dr h(r) int dL f(L; theta) eta(L / 4 pi r^2), with h(r) the
homogeneous distance density (Sec. 4.3) and eta the detection efficiency
of eq (5.10).  The oracle evaluates it with fixed Gauss-Legendre rules
(a 512-node rule in ln L over a precomputed efficiency table).  Pins:
  * its Gauss-Legendre nodes against numpy's leggauss;
  * the efficiency table against scipy adaptive quadrature of the defining
    integral over r (not the substituted form the oracle uses);
  * Z against nested scipy adaptive quadrature, against the Monte-Carlo
    detected fraction of the simulated population, and against the
    closed form of the zero-noise limit (a gamma-CDF expression);
  * node doubling (512 -> 1024) changes ln Z by < 1e-10.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import synth


@pytest.fixture(scope="module")
def lf_small():
    return synth.gamma_lf_1d(n=64, seed=11)


def _eps_scipy(x, fth, sigf, rmax):
    lum = math.exp(x)
    rstar = math.sqrt(lum / (4 * math.pi * fth))

    def integrand(r):
        flux = lum / (4 * math.pi * r * r)
        return 3 * r * r / rmax**3 * stats.norm.cdf((flux - fth) / sigf)

    pts = [rstar] if 0 < rstar < rmax else None
    val, _ = integrate.quad(integrand, 0.0, rmax, points=pts, limit=400, epsabs=1e-16, epsrel=1e-12)
    return val


@pytest.mark.parametrize("n", [5, 64, 512])
def test_gauss_legendre_matches_numpy(oracle_lib, n):
    x, w = oracle_lib.gauss_legendre(n, -2.0, 3.0)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, 0.5 + 2.5 * xr, rtol=0, atol=1e-13)
    # numpy's own weights carry ~1e-10 relative error at n = 512
    assert np.allclose(w, 2.5 * wr, rtol=5e-9, atol=1e-15)
    assert abs(w.sum() - 5.0) < 1e-12
    # exactness: the rule integrates P_j over [-1, 1] to zero for 1 <= j < 2n
    t = (x - 0.5) / 2.5
    for j in sorted({j for j in list(range(1, 12)) + [2 * n - 3, 2 * n - 1] if 1 <= j < 2 * n}):
        coef = np.zeros(j + 1)
        coef[j] = 1.0
        assert abs(np.dot(w / 2.5, np.polynomial.legendre.legval(t, coef))) < 1e-12


def test_efficiency_table_vs_scipy(oracle_lib, lf_small):
    o = oracle_lib.Oracle(lf_small)
    fth, sigf, rmax = lf_small.consts[0], lf_small.consts[1], lf_small.consts[2]
    lmax = 4 * math.pi * rmax**2 * fth
    for x in [math.log(lmax) - 12, math.log(lmax) - 3, math.log(lmax) - 0.5, math.log(lmax),
              math.log(lmax) + 0.3, math.log(lmax) + 3]:
        ref = _eps_scipy(x, fth, sigf, rmax)
        got = o.eps(x)
        # Far below Lmax the efficiency step sits where the fixed rule's nodes
        # are ~0.17 apart in t, so the relative error grows to ~1e-7 while the
        # absolute error stays < 1e-14 (what Z needs).
        assert got == pytest.approx(ref, rel=1e-6, abs=1e-14), x
    # below the threshold volume the efficiency follows (L/Lmax)^1.5
    x = math.log(lmax) - 6
    assert o.eps(x) == pytest.approx(math.exp(1.5 * (x - math.log(lmax))), rel=2e-2)


def test_Z_vs_nested_adaptive_quadrature(oracle_lib, lf_small):
    o = oracle_lib.Oracle(lf_small)
    fth, sigf, rmax = lf_small.consts[0], lf_small.consts[1], lf_small.consts[2]
    for beta, lnls in [(-0.3, math.log(5e10)), (-0.5, math.log(5e10) + 0.3), (-0.1, math.log(5e10) - 0.4)]:
        a = beta + 1.0

        def f_x(x):
            return math.exp(a * (x - lnls) - math.exp(x - lnls) - special.gammaln(a)) * _eps_scipy(x, fth, sigf, rmax)

        ref, _ = integrate.quad(f_x, lnls - 40.0, lnls + 5.0, limit=300, epsabs=1e-14, epsrel=1e-11)
        assert math.exp(o.log_Z([beta, lnls])) == pytest.approx(ref, rel=1e-8)


def test_Z_matches_monte_carlo_detection_fraction(oracle_lib, lf_small):
    o = oracle_lib.Oracle(lf_small)
    fth, rmax = lf_small.consts[0], lf_small.consts[2]
    rng = np.random.default_rng(2024)
    n = 4_000_000
    lum = rng.gamma(0.7, 5e10, n)
    r = rmax * rng.random(n) ** (1 / 3)
    fhat = lum / (4 * math.pi * r * r) + 0.1 * fth * rng.standard_normal(n)
    frac = np.mean(fhat > fth)
    z = math.exp(o.log_Z(lf_small.theta_true))
    se = math.sqrt(z * (1 - z) / n)
    assert abs(frac - z) < 4.5 * se
    assert abs(z - 0.3) < 0.01   # the generator calibrated F_th for a 30 % detected fraction


def test_Z_zero_noise_limit_closed_form(oracle_lib):
    wl = synth.gamma_lf_1d(n=16, seed=12)
    wl.consts[1] = 1e-4 * wl.consts[0]          # sigma_F -> 0: eta becomes a step
    o = oracle_lib.Oracle(wl)
    fth, rmax = wl.consts[0], wl.consts[2]
    lmax = 4 * math.pi * rmax**2 * fth
    for beta, lnls in [(-0.3, math.log(5e10)), (-0.7, math.log(3e10))]:
        a, ls = beta + 1.0, math.exp(lnls)
        c = lmax / ls
        # Z = P(L > Lmax) + Lmax^-1.5 E[L^1.5; L < Lmax] for L ~ Gamma(a, L*)
        ref = special.gammaincc(a, c) + (ls / lmax) ** 1.5 * math.exp(
            special.gammaln(a + 1.5) - special.gammaln(a)) * special.gammainc(a + 1.5, c)
        assert math.exp(o.log_Z([beta, lnls])) == pytest.approx(ref, rel=2e-2)


def test_Z_node_doubling(oracle_lib, lf_small):
    o512 = oracle_lib.Oracle(lf_small, nq=512)
    o1024 = oracle_lib.Oracle(lf_small, nq=1024)
    for th in [[-0.3, math.log(5e10)], [-0.45, math.log(5e10) + 0.2], [-0.2, math.log(5e10) - 0.2]]:
        assert abs(o512.log_Z(th) - o1024.log_Z(th)) < 1e-10
