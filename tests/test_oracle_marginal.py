"""Pins of the oracle's per-object marginal likelihood of 1-D latents (Sec. 6).

Sec. 6 proposes integrating each object's latent out by quadrature, which
leaves a likelihood of theta alone.  The oracle integrates l_i(chi) f(chi;
theta) over chi with composite Gauss-Legendre panels.  Its pins:

* normal-normal: the integral has a closed form (a normal of y with variance
  sigma^2 + tau^2);
* gamma LF: differences between two theta values against scipy's adaptive
  quadrature of an integrand written with scipy.stats (the member likelihood
  is defined up to a constant, which cancels in the difference);
* BB1: scipy's adaptive quadrature of the oracle's own pinned log terms,
  which checks the panels, including the far tail below the datum where the
  flux-dependent error keeps the member likelihood above zero;
* the marginal log-likelihood is the sum of the terms less N ln Z(theta).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import synth


@pytest.fixture(scope="module")
def nn1():
    oracle.build(force=False)
    return oracle.Oracle(synth.normal_normal_1d(n=200, seed=5))


@pytest.fixture(scope="module")
def lf1():
    oracle.build(force=False)
    return oracle.Oracle(synth.gamma_lf_1d(n=40, seed=23, fth=389.75))


@pytest.fixture(scope="module")
def bb1():
    oracle.build(force=False)
    return oracle.Oracle(synth.bb1_lf(n=40, seed=24, chunk=400_000))


def nn1d_closed_form(y, sig, mu, tau):
    # the member likelihood carries no constant: exp(-(y - chi)^2 / (2 sigma^2))
    v = sig * sig + tau * tau
    return np.log(sig / np.sqrt(v)) - (y - mu) ** 2 / (2.0 * v)


@pytest.mark.parametrize("theta", [[0.1, math.log(0.8)], [0.3, math.log(0.05)], [-2.0, math.log(30.0)],
                                   [5.0, math.log(1e-3)]])
def test_normal_normal_closed_form(nn1, theta):
    y, sig = nn1.wl.data
    got = nn1.marginal_terms(theta)
    ref = nn1d_closed_form(y, sig, theta[0], math.exp(theta[1]))
    assert np.max(np.abs(got - ref)) < 1e-12


def test_normal_normal_loglik_is_the_sum(nn1):
    th = [0.2, math.log(0.6)]
    assert nn1.marginal_loglik(th) == pytest.approx(float(np.sum(nn1.marginal_terms(th))), abs=1e-9)


def _lf1d_log_integral(fhat, k, sigf, beta, ln_lstar):
    # integrand in chi = ln L: N(fhat; F = e^(chi - k), sigf) times the gamma
    # density of L (shape beta + 1, scale e^ln_lstar) times the Jacobian L
    peak = math.log(fhat) + k
    w = sigf / fhat

    def g(x):
        return math.exp(stats.norm.logpdf(fhat, math.exp(x - k), sigf)
                        + stats.gamma.logpdf(math.exp(x), beta + 1.0, scale=math.exp(ln_lstar)) + x)
    pts = [peak - 300, peak - 40 * w, peak - 8 * w, peak, peak + 8 * w, peak + 40 * w, peak + 15]
    pts = sorted(set(pts))
    s = sum(integrate.quad(g, a, b, limit=400, epsabs=0, epsrel=1e-12)[0] for a, b in zip(pts, pts[1:]))
    return math.log(s)


def test_gamma_lf_differences_match_adaptive_quadrature(lf1):
    fhat, k = lf1.wl.data.astype(np.float64)
    sigf = lf1.wl.consts[1]
    ta = np.array(lf1.wl.theta_true, dtype=np.float64)
    tb = ta + np.array([0.15, -0.4])
    da = lf1.marginal_terms(ta) - lf1.marginal_terms(tb)
    for i in (0, 5, 17, 39):
        ref = (_lf1d_log_integral(fhat[i], k[i], sigf, *ta) - _lf1d_log_integral(fhat[i], k[i], sigf, *tb))
        assert abs(da[i] - ref) < 1e-10, i


def _quad_of_log_terms(o, i, theta):
    fhat, k = float(o.wl.data[0][i]), float(o.wl.data[1][i])
    peak = math.log(fhat) + k
    shift = sum(o.log_terms(i, [peak], theta))

    def g(x):
        return math.exp(sum(o.log_terms(i, [x], theta)) - shift)
    pts = [peak - 400, peak - 60, peak - 10, peak - 1, peak - 0.2, peak, peak + 0.2, peak + 1, peak + 15]
    return shift + math.log(sum(integrate.quad(g, a, b, limit=400, epsabs=0, epsrel=1e-13)[0]
                                for a, b in zip(pts, pts[1:])))


@pytest.mark.parametrize("theta", [[-1.5, math.log(0.01), 0.0], [-1.2, math.log(0.05), math.log(2.0)],
                                   [-0.5, math.log(0.002), math.log(0.5)]])
def test_bb1_terms_match_adaptive_quadrature(bb1, theta):
    got = bb1.marginal_terms(theta)
    for i in (0, 3, 11, 29):
        assert abs(got[i] - _quad_of_log_terms(bb1, i, theta)) < 1e-10, i


def test_bb1_tail_below_the_datum_counts(bb1):
    """With sigma(F) -> sigma0 as F -> 0 the member likelihood of a faint
    detection stays at about exp(-nu^2/2) of its peak far below the datum; the
    population mass there must enter the integral."""
    th = [-1.5, math.log(0.01), 0.0]
    fhat = bb1.wl.data[0]
    i = int(np.argmin(fhat))
    full = _quad_of_log_terms(bb1, i, th)
    k = float(bb1.wl.data[1][i])
    peak = math.log(float(fhat[i])) + k
    shift = sum(bb1.log_terms(i, [peak], th))
    near = shift + math.log(integrate.quad(lambda x: math.exp(sum(bb1.log_terms(i, [x], th)) - shift),
                                           peak - 3, peak + 15, limit=400, epsrel=1e-13)[0])
    assert full - near > 1e-7           # the tail is not negligible at this tolerance
    assert abs(bb1.marginal_terms(th)[i] - full) < 1e-10


def test_selection_enters_the_loglik(lf1):
    th = lf1.wl.theta_true
    assert lf1.marginal_loglik(th) == pytest.approx(float(np.sum(lf1.marginal_terms(th))) - lf1.n * lf1.log_Z(th),
                                                    abs=1e-8)


def test_three_d_latents_are_refused():
    o = oracle.Oracle(synth.normal_normal_3d(n=8))
    with pytest.raises(ValueError):
        o.marginal_terms([0.0, 0.0, 0.0])


def test_bb1_slow_power_tail(bb1):
    """Near beta = -2 the luminosity PDF falls only as L^(beta + 2) below l:
    the integral reaches hundreds of e-folds below the datum."""
    th = [-1.95, math.log(0.01), 0.0]
    got = bb1.marginal_terms(th)
    for i in (0, 11):
        fhat, k = float(bb1.wl.data[0][i]), float(bb1.wl.data[1][i])
        peak = math.log(fhat) + k
        shift = sum(bb1.log_terms(i, [peak], th))
        g = lambda x: math.exp(sum(bb1.log_terms(i, [x], th)) - shift)
        pts = [peak - 60, peak - 10, peak - 1, peak, peak + 1, peak + 15]
        v = integrate.quad(g, -np.inf, pts[0], limit=400, epsabs=0, epsrel=1e-12)[0]
        v += sum(integrate.quad(g, a, b, limit=400, epsabs=0, epsrel=1e-13)[0] for a, b in zip(pts, pts[1:]))
        assert abs(got[i] - (shift + math.log(v))) < 1e-9, i
