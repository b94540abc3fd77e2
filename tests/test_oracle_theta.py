"""Pins for the oracle's population-parameter step and the whole MWG sampler.

The sampler reaches a distribution, so these pins compare chain moments
(batch-means Monte Carlo standard errors) with posteriors computed another
way:
  * theta | chi of the normal-normal model has closed-form conditionals
    (mu | tau, chi ~ N(mean chi, tau^2/N); tau has density
    tau^{-(N-2)} exp(-SS / 2 tau^2) in ln tau under a uniform-tau prior);
  * the full normal-normal posterior p(mu, tau | y) is proportional to
    tau prod_i N(y_i; mu, tau^2 + sigma_i^2), evaluated on a 2-D grid;
  * the paper's 3-D normal-normal instance (Sec. 3) with a flat prior on
    mu has mu | y ~ N(mean y, (C_pop + diag sigma^2) / N);
  * a tiny luminosity-function catalog is solved by brute force: a theta
    grid times per-object 1-D integrals over chi times Z(theta)^-N, with Z
    from an independent scipy evaluation of its defining integral;
  * the theta proposal factor obeys the RAM determinant identity.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import synth
from conftest import batch_means

TOL_MCSE = 3.0


def _check(chain, ref_mean, ref_var, label):
    m, se = batch_means(chain)
    assert abs(m - ref_mean) < TOL_MCSE * se, (label, m, ref_mean, se)
    dv, se_v = batch_means((chain - ref_mean) ** 2)
    assert abs(dv - ref_var) < TOL_MCSE * se_v + 1e-12, (label, dv, ref_var, se_v)


@pytest.mark.parametrize("n", [1000, 40])
def test_theta_given_chi_closed_form(oracle_lib, n):
    wl = synth.normal_normal_1d(n=n, seed=0)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    st.chi[0] = wl.truth["chi"]                        # condition on a fixed latent state
    tt, _ = o.run(st, 60000, fix_chi=True)
    keep = tt[5000:]
    chi = wl.truth["chi"]
    n, xbar, ss = chi.size, chi.mean(), np.sum((chi - chi.mean()) ** 2)
    lt = np.linspace(-2.0, 2.0, 400001)
    logp = -(n - 2) * lt - ss / (2 * np.exp(2 * lt))
    p = np.exp(logp - logp.max())
    p /= np.trapezoid(p, lt)
    e_lt = np.trapezoid(lt * p, lt)
    v_lt = np.trapezoid((lt - e_lt) ** 2 * p, lt)
    e_tau2 = np.trapezoid(np.exp(2 * lt) * p, lt)
    _check(keep[:, 0], xbar, e_tau2 / n, "mu")
    _check(keep[:, 1], e_lt, v_lt, "ln tau")


def test_normal_normal_full_posterior_grid(oracle_lib):
    wl = synth.normal_normal_1d(n=1000, seed=0)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    tt, _ = o.run(st, 60000)
    keep = tt[10000:]
    y, sig = wl.data
    mu = np.linspace(-0.35, 0.2, 221)
    lt = np.linspace(-0.35, 0.2, 221)
    M, LT = np.meshgrid(mu, lt, indexing="ij")
    logp = LT.copy()
    var = np.exp(2 * LT)[..., None] + sig**2
    logp += np.sum(-0.5 * np.log(var) - 0.5 * (y - M[..., None]) ** 2 / var, axis=-1)
    p = np.exp(logp - logp.max())
    p /= p.sum()
    for idx, grid in ((0, M), (1, LT)):
        mean = np.sum(p * grid)
        varr = np.sum(p * (grid - mean) ** 2)
        _check(keep[:, idx], mean, varr, f"theta[{idx}]")


def test_papers_3d_normal_normal_closed_form(oracle_lib):
    wl = synth.normal_normal_3d(n=1000, seed=5)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    tt, _ = o.run(st, 30000)
    keep = tt[6000:]
    cpop = np.diag(synth.workloads.NN3D_D) @ synth.workloads.NN3D_R @ np.diag(synth.workloads.NN3D_D)
    cov = (cpop + np.diag(synth.workloads.NN3D_SIGMA**2)) / wl.n
    ybar = wl.data.mean(axis=1)
    for j in range(3):
        _check(keep[:, j], ybar[j], cov[j, j], f"mu[{j}]")
    # latent factors adapt towards the per-object conditional covariance shape
    post = np.linalg.inv(np.linalg.inv(cpop) + np.diag(1 / synth.workloads.NN3D_SIGMA**2))
    s = np.zeros((3, 3))
    e = 0
    for r in range(3):
        for c in range(r + 1):
            s[r, c] = np.median(st.chol[e])
            e += 1
    corr = lambda a: a / np.sqrt(np.outer(np.diag(a), np.diag(a)))  # noqa: E731
    assert np.allclose(corr(s @ s.T), corr(post), atol=0.15)


@pytest.mark.slow
def test_tiny_catalog_brute_force(oracle_lib):
    wl = synth.gamma_lf_1d(n=12, seed=41, fth=389.75)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    tt, _ = o.run(st, 150000)
    keep = tt[30000:]
    fhat, k = wl.data.astype(np.float64)
    fth, sigf, rmax = wl.consts[0], wl.consts[1], wl.consts[2]

    # Efficiency eps(ln L) from the defining integral over r (scipy), then
    # Z(theta) by the trapezoid rule on a fine ln L grid.
    def eps(x):
        lum = math.exp(x)

        def f(r):
            return 3 * r * r / rmax**3 * stats.norm.cdf((lum / (4 * math.pi * r * r) - fth) / sigf)
        rs = math.sqrt(lum / (4 * math.pi * fth))
        return integrate.quad(f, 0, rmax, points=[rs] if rs < rmax else None, limit=200)[0]

    xg = np.linspace(math.log(5e10) - 25, math.log(5e10) + 4, 700)
    epsg = np.array([eps(x) for x in xg])
    beta = np.linspace(-0.995, -0.005, 100)
    lnls = np.linspace(math.log(5e10) - 4, math.log(5e10) + 4, 161)
    B, LS = np.meshgrid(beta, lnls, indexing="ij")
    a = (B + 1)[..., None]

    def logf(x):
        return a * (x - LS[..., None]) - np.exp(x - LS[..., None]) - special.gammaln(a)

    logz = np.log(np.trapezoid(np.exp(logf(xg)) * epsg, xg, axis=-1))
    logp = -np.log1p(B**2) - wl.n * logz
    for i in range(wl.n):
        c0 = k[i] + math.log(fhat[i])
        w = 6 * sigf / fhat[i]
        xs = np.linspace(c0 - w, c0 + w, 801)
        lm = -0.5 * ((fhat[i] - np.exp(xs - k[i])) / sigf) ** 2
        integ = np.trapezoid(np.exp(logf(xs) + lm), xs, axis=-1)
        logp += np.log(integ)
    p = np.exp(logp - logp.max())
    p /= p.sum()
    for idx, grid in ((0, B), (1, LS)):
        mean = np.sum(p * grid)
        varr = np.sum(p * (grid - mean) ** 2)
        _check(keep[:, idx], mean, varr, f"theta[{idx}]")


def test_theta_factor_determinant_identity(oracle_lib):
    wl = synth.gamma_lf_1d(n=300, seed=42)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    o.run(st, 20)
    for _ in range(5):
        o.sweep(st)
        before = st.chol_theta.copy()
        info = o.theta_step(st)
        eta = (st.k + 1) ** (-2 / 3)
        c = eta * (info["alpha"] - 0.4)
        ld = np.sum(np.log(np.diag(st.chol_theta))) - np.sum(np.log(np.diag(before)))
        assert ld == pytest.approx(0.5 * math.log1p(c), rel=1e-10, abs=1e-14)
        z = np.array([oracle_lib.variates(wl.seed, [0, st.k, 1, j // 4])[1][j % 4] for j in range(2)])
        tgt = before @ (np.eye(2) + c * np.outer(z, z) / z.dot(z)) @ before.T
        np.testing.assert_allclose(st.chol_theta, np.linalg.cholesky(tgt), rtol=1e-12, atol=1e-15)


def test_theta_substeps_sample_theta_given_chi(oracle_lib):
    """Several Metropolis steps on theta per cycle (each from the full N-term
    sums) still sample theta | chi: the normal-normal closed form."""
    wl = synth.normal_normal_1d(n=200, seed=0)
    o = oracle_lib.Oracle(wl, theta_substeps=3)
    st = o.initial_state()
    chi = wl.truth["chi"]
    st.chi[0] = chi
    tt, _ = o.run(st, 25000, fix_chi=True)
    keep = tt[2500:]
    n, xbar, ss = chi.size, chi.mean(), np.sum((chi - chi.mean()) ** 2)
    lt = np.linspace(-2.0, 2.0, 400001)
    logp = -(n - 2) * lt - ss / (2 * np.exp(2 * lt))
    p = np.exp(logp - logp.max())
    p /= np.trapezoid(p, lt)
    e_lt = np.trapezoid(lt * p, lt)
    v_lt = np.trapezoid((lt - e_lt) ** 2 * p, lt)
    e_tau2 = np.trapezoid(np.exp(2 * lt) * p, lt)
    _check(keep[:, 0], xbar, e_tau2 / n, "mu")
    _check(keep[:, 1], e_lt, v_lt, "ln tau")


def _ram_factor(low, z, c):
    # lower factor of S (I + c z z^T / |z|^2) S^T
    m = low @ (np.eye(len(z)) + c * np.outer(z, z) / (z @ z)) @ low.T
    return np.linalg.cholesky(m)


def test_theta_substep_draws_and_adaptation(oracle_lib):
    """Sub-step j of cycle k draws from Philox blocks (j, k, 1, b) and
    (j, k, 2, 0) and adapts with eta_n, n = (k - 1) K + j + 1."""
    wl = synth.gamma_lf_1d(n=60, seed=31, fth=389.75)
    K, gamma = 2, 2.0 / 3.0
    o = oracle_lib.Oracle(wl, theta_substeps=K)
    st = o.initial_state()
    o.run(st, 4)
    k = st.k + 1
    theta, low = st.theta.copy(), st.chol_theta.copy()
    st.k = k
    n_acc = 0
    for j in range(K):
        z = np.array([oracle_lib.variates(o.seed, [j, k, 1, r // 4])[1][r % 4] for r in range(o.p)])
        prop = theta + low @ z
        lp = o.log_prior(prop)
        delta = -math.inf
        if np.isfinite(lp):
            delta = (lp + o.pop_sum(prop, st.chi) - o.n * o.log_Z(prop)) - \
                    (o.log_prior(theta) + o.pop_sum(theta, st.chi) - o.n * o.log_Z(theta))
        ln_u = math.log(oracle_lib.variates(o.seed, [j, k, 2, 0])[0][4])
        alpha = 1.0 if delta >= 0 else math.exp(delta)
        if ln_u < delta:
            theta, n_acc = prop, n_acc + 1
        eta = ((k - 1) * K + j + 2) ** -gamma
        low = _ram_factor(low, z, eta * (alpha - 0.4))
    info = o.theta_step(st)
    assert info["n_accepted"] == n_acc
    assert np.allclose(st.theta, theta, rtol=0, atol=1e-12)
    assert np.allclose(st.chol_theta, low, rtol=1e-10, atol=1e-13)
