"""Pins of the oracle's break-by-one (BB1) luminosity-function model (Sec. 5, Appendix C).

Each check compares the oracle with something fixed independently of it:
the normalisation of a PDF, the gamma law BB1 reduces to as l -> 0, the
closed-form CDF of Appendix C (read with the lower incomplete gamma
function), the member likelihood as a normal sampling density, adaptive
quadrature of the detection efficiency, and a Monte Carlo detection fraction
for the selection normaliser.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
import synth


@pytest.fixture(scope="module")
def wl():
    return synth.bb1_lf(n=400, seed=11, chunk=1_000_000)


@pytest.fixture(scope="module")
def orc(wl):
    oracle.build(force=False)
    return oracle.Oracle(wl)


def _pop(orc, x, theta):
    return orc.log_terms(0, [x], theta)[1]


def _integral_over_x(fn):
    # the PDF falls only as L^(beta + 2) below l: start far out
    pts = [-500, -200, -60, -20, -10, -5, -2, 0, 2, 5]
    return sum(integrate.quad(fn, a, b, limit=400, epsabs=0, epsrel=1e-12)[0] for a, b in zip(pts, pts[1:]))


@pytest.mark.parametrize("beta", [-1.5, -1.9, -1.0, -1.0 + 1e-7, -0.5, -0.05])
@pytest.mark.parametrize("ln_l,ln_u", [(math.log(0.01), 0.0), (math.log(0.3), math.log(2.0))])
def test_population_density_integrates_to_one(orc, beta, ln_l, ln_u):
    theta = [beta, ln_l, ln_u]
    total = _integral_over_x(lambda x: math.exp(_pop(orc, x, theta)))
    assert abs(total - 1.0) < 1e-8


def test_continuous_at_beta_minus_one(orc):
    x, ln_l, ln_u = -1.3, math.log(0.01), 0.0
    at = _pop(orc, x, [-1.0, ln_l, ln_u])
    for eps in (1e-6, -1e-6):
        assert abs(_pop(orc, x, [-1.0 + eps, ln_l, ln_u]) - at) < 1e-5


@pytest.mark.parametrize("beta", [-0.7, -0.3])
def test_small_break_reduces_to_gamma(orc, beta):
    # l -> 0: (1 - e^{-L/l}) -> 1 and C -> 1 / Gamma(beta + 1) (slowly: the
    # correction to C is (1 + u/l)^-(beta+1))
    ln_u = math.log(1.7)
    for x in (-3.0, 0.0, 1.2):
        ref = stats.gamma.logpdf(math.exp(x), beta + 1.0, scale=1.7) + x
        assert abs(_pop(orc, x, [beta, math.log(1e-60), ln_u]) - ref) < 1e-9


@pytest.mark.parametrize("beta", [-0.8, -0.3])
def test_cdf_of_appendix_c(orc, beta):
    l, u = 0.05, 1.3
    theta = [beta, math.log(l), math.log(u)]
    lnc = oracle.bb1_log_norm(beta, math.log(l), math.log(u))
    a = beta + 1.0
    lower = lambda s, z: special.gammainc(s, z) * special.gamma(s)   # unregularised lower incomplete gamma
    for L in (0.02, 0.4, 2.0):
        cdf = math.exp(lnc) * (lower(a, L / u) - lower(a, L * (1 / u + 1 / l)) / (1 + u / l) ** a)
        num = integrate.quad(lambda x: math.exp(_pop(orc, x, theta)), -60, math.log(L), limit=400,
                             epsabs=0, epsrel=1e-12)[0]
        assert abs(num - cdf) < 1e-9


def test_member_likelihood_is_the_sampling_density(orc, wl):
    th = wl.theta_true
    s0, alpha = wl.consts[1], wl.consts[2]
    for i in (0, 7, 99):
        fhat, k = float(wl.data[0][i]), float(wl.data[1][i])
        vals = []
        for x in (k + math.log(fhat) - 0.05, k + math.log(fhat), k + math.log(fhat) + 0.2):
            flux = math.exp(x - k)
            ref = stats.norm.logpdf(fhat, flux, math.sqrt(s0 ** 2 + (alpha * flux) ** 2)) + 0.5 * math.log(2 * math.pi)
            vals.append(orc.log_terms(i, [x], th)[0] - ref)
        assert max(abs(v) for v in vals) < 1e-12


@pytest.mark.parametrize("x", [math.log(0.5), math.log(3.0), math.log(20.0), math.log(200.0)])
def test_efficiency_by_adaptive_quadrature(orc, wl, x):
    fth, s0, alpha = wl.consts[0], wl.consts[1], wl.consts[2]
    lum = math.exp(x)

    def integrand(r):
        flux = lum / (r * r)
        return 3 * r * r * stats.norm.cdf((flux - fth) / math.sqrt(s0 ** 2 + (alpha * flux) ** 2))
    r_th = math.sqrt(lum / fth)
    pts = [p for p in (0.5 * r_th, r_th, 1.5 * r_th) if p < 1.0]
    ref = integrate.quad(integrand, 0, 1, points=pts or None, limit=400, epsabs=1e-15, epsrel=1e-11)[0]
    assert abs(orc.eps(x) - ref) <= 1e-7 * ref + 1e-13


@pytest.mark.parametrize("theta", [[-1.5, math.log(0.01), 0.0], [-1.2, math.log(0.02), math.log(1.5)]])
def test_selection_normaliser_matches_monte_carlo(orc, theta):
    rng = np.random.default_rng(17)
    m = 8_000_000
    lum = synth.bb1_sample(rng, m, theta[0], math.exp(theta[1]), math.exp(theta[2]))
    r = rng.random(m) ** (1.0 / 3.0)
    flux = lum / (r * r)
    s0, alpha, fth = orc.wl.consts[1], orc.wl.consts[2], orc.wl.consts[0]
    fhat = flux + np.sqrt(s0 ** 2 + (alpha * flux) ** 2) * rng.standard_normal(m)
    p = np.count_nonzero(fhat > fth) / m
    z = math.exp(orc.log_Z(theta))
    assert abs(z - p) < 4.5 * math.sqrt(p * (1 - p) / m)


def test_prior_of_eq_5_5(orc):
    # p(beta) ~ 1/(1+beta^2) on (-2, 0), flat in l, flat in ln u, l < u:
    # as a density in (beta, ln l, ln u) that is l / (1 + beta^2)
    a, b = [-1.5, math.log(0.01), 0.0], [-0.4, math.log(0.2), math.log(3.0)]
    got = orc.log_prior(b) - orc.log_prior(a)
    ref = (math.log(0.2) - math.log(1 + 0.16)) - (math.log(0.01) - math.log(1 + 2.25))
    assert abs(got - ref) < 1e-13
    for bad in ([-2.0, -3.0, 0.0], [0.0, -3.0, 0.0], [-1.0, 0.5, 0.4]):
        assert orc.log_prior(bad) == -math.inf


def test_theta_step_includes_selection(wl):
    o = oracle.Oracle(wl)
    st = o.initial_state()
    o.run(st, 20)
    cur = st.theta.copy()
    st.k += 1
    prop = o.theta_proposal(st, k=st.k)
    info = o.theta_step(st)
    ref = (o.log_prior(prop) + o.pop_sum(prop, st.chi) - wl.n * o.log_Z(prop)) - \
          (o.log_prior(cur) + o.pop_sum(cur, st.chi) - wl.n * o.log_Z(cur))
    if math.isfinite(ref):
        assert abs(info["delta"] - ref) < 1e-8
    else:
        assert info["delta"] == -math.inf


def test_generator_sampler_matches_the_density():
    rng = np.random.default_rng(3)
    x = np.log(synth.bb1_sample(rng, 400_000, -1.5, 0.01, 1.0))
    o = oracle.Oracle(synth.bb1_lf(n=10, seed=1, chunk=200_000))
    grid = np.linspace(-12, 2.5, 60)
    cdf_num = np.array([np.mean(x <= g) for g in grid])
    th = [-1.5, math.log(0.01), 0.0]
    cdf_ref = np.array([integrate.quad(lambda t: math.exp(_pop(o, t, th)), -60, g, limit=300)[0] for g in grid])
    assert np.max(np.abs(cdf_num - cdf_ref)) < 4.0 / math.sqrt(400_000) * 2
