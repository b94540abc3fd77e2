"""Pins for the oracle's member likelihoods, population densities and priors.

Population densities are pinned by library routines (scipy.stats) and by
their normalisation (they must integrate to one in the latent coordinates;
the luminosity PDF carries the Jacobian of chi = ln L).  Member likelihoods
are defined up to a constant (Sec. 2.1), so they are pinned through
differences between two latent values.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import synth


@pytest.fixture(scope="module")
def models(oracle_lib):
    return {
        "nn1": oracle_lib.Oracle(synth.normal_normal_1d(n=50)),
        "lf1": oracle_lib.Oracle(synth.gamma_lf_1d(n=50, seed=21)),
        "lf3": oracle_lib.Oracle(synth.gamma_lf_3d(n=50, seed=22)),
        "nn3": oracle_lib.Oracle(synth.normal_normal_3d(n=50)),
    }


def test_nn1d_terms(models):
    o = models["nn1"]
    y, sig = o.wl.data
    rng = np.random.default_rng(1)
    for _ in range(20):
        i = int(rng.integers(0, o.n))
        th = np.array([rng.normal(), rng.normal(0, 0.5)])
        x1, x2 = rng.normal(0, 2, 2)
        lm1, lp1 = o.log_terms(i, [x1], th)
        lm2, _ = o.log_terms(i, [x2], th)
        assert lp1 == pytest.approx(stats.norm.logpdf(x1, th[0], math.exp(th[1])), rel=1e-13)
        assert lm1 - lm2 == pytest.approx(stats.norm.logpdf(y[i], x1, sig[i]) - stats.norm.logpdf(y[i], x2, sig[i]),
                                          rel=1e-12, abs=1e-12)
    # prior: flat in mu, uniform in tau -> density tau in (mu, ln tau)
    assert o.log_prior([0.3, 0.7]) - o.log_prior([-2.0, 0.2]) == pytest.approx(0.5)


def test_lf1d_population_density_is_gamma_in_log_space(models):
    o = models["lf1"]
    for beta, lnls in [(-0.3, math.log(5e10)), (-0.8, math.log(1e10)), (-0.05, math.log(9e10))]:
        for x in [lnls - 6, lnls - 1, lnls, lnls + 1.5]:
            _, lp = o.log_terms(0, [x], [beta, lnls])
            ref = stats.gamma.logpdf(math.exp(x), beta + 1, scale=math.exp(lnls)) + x
            assert lp == pytest.approx(ref, rel=1e-12)
        norm, _ = integrate.quad(lambda x: math.exp(o.log_terms(0, [x], [beta, lnls])[1]),
                                 lnls - 250, lnls + 6, limit=400)
        assert norm == pytest.approx(1.0, abs=1e-9)


def test_lf1d_member_likelihood(models):
    o = models["lf1"]
    fhat, k = o.wl.data.astype(np.float64)
    sigf = o.wl.consts[1]
    th = o.wl.theta_true
    for i in range(10):
        x1, x2 = o.wl.chi0[0, i] + 0.01, o.wl.chi0[0, i] - 0.03
        lm1, _ = o.log_terms(i, [x1], th)
        lm2, _ = o.log_terms(i, [x2], th)
        ref = (stats.norm.logpdf(fhat[i], math.exp(x1 - k[i]), sigf)
               - stats.norm.logpdf(fhat[i], math.exp(x2 - k[i]), sigf))
        assert lm1 - lm2 == pytest.approx(ref, rel=1e-9, abs=1e-9)


def test_lf1d_prior_support(models):
    o = models["lf1"]
    assert o.log_prior([-0.3, 20.0]) == pytest.approx(-math.log(1.09))
    for bad in ([-1.0, 24.0], [0.0, 24.0], [0.2, 24.0], [-1.5, 24.0]):
        assert o.log_prior(bad) == -math.inf


def test_lf3d_terms(models):
    o = models["lf3"]
    fhat, rhat, chat = o.wl.data.astype(np.float64)
    sigf, rmax, sigr, sigc = o.wl.consts[1], o.wl.consts[2], o.wl.consts[4], o.wl.consts[5]
    th = np.array([-0.35, math.log(4e10), -1.8, 0.09, 0.25])
    for i in range(8):
        x = o.wl.chi0[:, i] + np.array([0.02, -0.01, 0.03])
        x[1] = min(x[1], math.log(rmax) - 1e-6)
        lm, lp = o.log_terms(i, x, th)
        ref_pop = (stats.gamma.logpdf(math.exp(x[0]), th[0] + 1, scale=math.exp(th[1])) + x[0]
                   + math.log(3 * math.exp(3 * x[1]) / rmax**3)
                   + stats.norm.logpdf(x[2], th[2] + th[3] * x[0], th[4]))
        assert lp == pytest.approx(ref_pop, rel=1e-12)
        x2 = x - np.array([0.01, 0.005, -0.02])
        lm2, _ = o.log_terms(i, x2, th)

        def meas(v):
            flux = math.exp(v[0]) / (4 * math.pi * math.exp(2 * v[1]))
            return (stats.norm.logpdf(fhat[i], flux, sigf) + stats.norm.logpdf(rhat[i], math.exp(v[1]), sigr * rhat[i])
                    + stats.norm.logpdf(chat[i], v[2], sigc))

        assert lm - lm2 == pytest.approx(meas(x) - meas(x2), rel=1e-8, abs=1e-8)
    # the distance part is a normalised density in ln r on (-inf, ln rmax], zero beyond
    norm, _ = integrate.quad(lambda u: math.exp(o.log_terms(0, [25.0, u, 0.5], [-0.3, 25.0, 0.0, 0.0, 1.0])[1]
                                                - o.log_terms(0, [25.0, math.log(rmax) - 1.0, 0.5],
                                                              [-0.3, 25.0, 0.0, 0.0, 1.0])[1]
                                                + math.log(3 * math.exp(3 * (math.log(rmax) - 1.0)) / rmax**3)),
                             math.log(rmax) - 30, math.log(rmax))
    assert norm == pytest.approx(1.0, abs=1e-9)
    _, lp_out = o.log_terms(0, [25.0, math.log(rmax) + 1e-6, 0.5], th)
    assert lp_out == -math.inf
    assert o.log_prior([-0.3, 24.0, 0.0, 0.0, -0.1]) == -math.inf
    assert o.log_prior([-0.3, 24.0, 0.0, 0.0, 0.1]) == pytest.approx(-math.log(1.09))


def test_nn3d_population_is_the_papers_mvn(models):
    o = models["nn3"]
    cpop = np.diag(synth.workloads.NN3D_D) @ synth.workloads.NN3D_R @ np.diag(synth.workloads.NN3D_D)
    rng = np.random.default_rng(3)
    for _ in range(10):
        x = rng.normal(0, 3, 3)
        mu = rng.normal(0, 1, 3)
        _, lp = o.log_terms(0, x, mu)
        assert lp == pytest.approx(stats.multivariate_normal.logpdf(x, mu, cpop), rel=1e-12)
