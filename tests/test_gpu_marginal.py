"""GPU parity of the marginal likelihood of 1-D latents (Sec. 6).

The device integrates each object's latent out with its own FP64 rule
(flux-space core, graded panels below the datum, a power-law tail); the
oracle integrates the same integrand with fine composite panels.  Checks:

* per-object log integrals against the oracle, element by element, at sizes
  that span several workgroups with a ragged tail, for the normal-normal,
  gamma-LF and BB1 models at theta in the posterior bulk and far from it;
* the latent-free log-likelihood (sum less N ln Z) against the oracle's;
* at the full size of the single-GPU gamma-LF catalog (N = 300000): sampled
  objects against the oracle, and the sum of the per-object terms;
* a batch of theta rows equals the rows evaluated one by one, bitwise, and a
  slot of a batch equals the same catalog alone;
* random-walk Metropolis on theta over the marginal likelihood reaches the
  posterior the Metropolis-within-Gibbs sampler reaches (an independent
  cross-check of the sampled latents);
* argument errors.

Tolerance: 1e-9 absolute per object.  The rule's own error, measured against
the oracle over the theta used here, is below 7e-11; FP64 rounding of a
216-node sum adds ~1e-14 per term.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import MOMENT_BATCHES, batch_means

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TERM_TOL = 1e-9


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2105_08026_amd as h
    h.lib()
    return h


def _subset(wl, idx):
    import copy
    w = copy.copy(wl)
    w.data = np.ascontiguousarray(wl.data[:, idx])
    w.chi0 = np.ascontiguousarray(wl.chi0[:, idx])
    w.n = len(idx)
    return w


def _thetas(wl):
    t0 = np.array(wl.theta_true, dtype=np.float64)
    if wl.model == synth.NormalNormal1D:
        return [t0, [0.3, math.log(0.05)], [-2.0, math.log(30.0)], [5.0, math.log(1e-3)]]
    if wl.model == synth.GammaLF1D:
        return [t0, t0 + [0.05, -0.1], [-0.9, t0[1] + 1.0], [-0.05, t0[1] - 1.5], [-0.5, t0[1] - 3.0]]
    return [t0, t0 + [0.1, 0.2, -0.1], [-1.2, t0[1] + 0.5, t0[2] + 0.2], [-0.1, t0[1] + 1.0, t0[2] - 0.3],
            [-1.8, t0[1] - 1.0, t0[2] + 0.5], [-1.5, t0[1], t0[2] - 2.0], [-1.95, t0[1], t0[2]]]


WORKLOADS = {
    "nn1d": lambda n: synth.normal_normal_1d(n=n, seed=71),
    "lf1d": lambda n: synth.gamma_lf_1d(n=n, seed=72, fth=389.75),
    "bb1": lambda n: synth.bb1_lf(n=n, seed=73, chunk=1_000_000),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("n", [3001, 31])
def test_terms_match_oracle(hbm, name, n):
    wl = WORKLOADS[name](n)
    _say(f"marginal terms {name} N={n}")
    s = hbm.Sampler(wl, max_cycles=4)
    o = oracle.Oracle(wl)
    ths = np.array(_thetas(wl), dtype=np.float64)
    out, terms = s.marginal_loglik(ths, terms=True)
    for j, th in enumerate(ths):
        ref = o.marginal_terms(th)
        err = np.max(np.abs(terms[j] - ref))
        _say(f"  theta {np.round(th, 3)}: max |term - oracle| = {err:.2e}")
        assert err < TERM_TOL, (j, err)
        # the total: the terms' sum less N ln Z (the device's selection
        # quadrature agrees with the oracle's to ~1e-9 in ln Z)
        tot_ref = o.marginal_loglik(th)
        assert abs(out[j] - tot_ref) <= (TERM_TOL + 1e-8) * wl.n, (j, out[j], tot_ref)
    s.close()


def test_full_size_gamma_lf_sampled(hbm):
    wl = synth.gamma_lf_1d(n=300_000, seed=1)
    _say(f"marginal full size gamma LF N={wl.n}")
    s = hbm.Sampler(wl, max_cycles=4)
    th = np.array(wl.theta_true, dtype=np.float64)
    out, terms = s.marginal_loglik(th, terms=True)
    rng = np.random.default_rng(5)
    idx = np.sort(np.concatenate([rng.choice(wl.n, 1500, replace=False), np.arange(wl.n - 40, wl.n)]))
    o = oracle.Oracle(_subset(wl, idx))
    ref = o.marginal_terms(th)
    err = np.max(np.abs(terms[0][idx] - ref))
    _say(f"  sampled {len(idx)} objects: max |term - oracle| = {err:.2e}")
    assert err < TERM_TOL
    # the device's fixed-order FP64 sum against an exact sum of its own terms
    lz = oracle.Oracle(_subset(wl, idx[:8])).log_Z(th)
    assert abs(out[0] + wl.n * lz - math.fsum(terms[0])) <= 1e-8 * wl.n
    assert np.all(np.isfinite(terms[0]))
    s.close()


def test_full_size_bb1_sampled(hbm):
    wl = synth.bb1_lf(n=100_000)
    _say(f"marginal full size BB1 N={wl.n}")
    s = hbm.Sampler(wl, max_cycles=4)
    th = np.array(wl.theta_true, dtype=np.float64)
    out, terms = s.marginal_loglik(th, terms=True)
    rng = np.random.default_rng(6)
    idx = np.sort(np.concatenate([rng.choice(wl.n, 600, replace=False), np.arange(wl.n - 40, wl.n)]))
    ref = oracle.Oracle(_subset(wl, idx)).marginal_terms(th)
    err = np.max(np.abs(terms[0][idx] - ref))
    _say(f"  sampled {len(idx)} objects: max |term - oracle| = {err:.2e}")
    assert err < TERM_TOL
    assert np.all(np.isfinite(terms[0]))
    s.close()


def test_theta_rows_are_independent_and_deterministic(hbm):
    wl = synth.bb1_lf(n=5000, seed=74, chunk=1_000_000)
    s = hbm.Sampler(wl, max_cycles=4)
    ths = np.array(_thetas(wl), dtype=np.float64)
    together = s.marginal_loglik(ths)
    again = s.marginal_loglik(ths)
    one_by_one = np.array([s.marginal_loglik(th)[0] for th in ths])
    assert np.array_equal(together, again)
    assert np.array_equal(together, one_by_one)
    s.close()


def test_batch_slot_equals_alone(hbm):
    wls = [synth.gamma_lf_1d(n=n, seed=75 + j, fth=389.75) for j, n in enumerate((900, 2100))]
    b = hbm.Batch(wls, max_cycles=4)
    for j, w in enumerate(wls):
        th = np.array([w.theta_true, np.array(w.theta_true) + [0.02, 0.1]])
        s = hbm.Sampler(w, max_cycles=4)
        assert np.array_equal(b.marginal_loglik(j, th), s.marginal_loglik(th)), j
        s.close()
    b.close()


def _rw_metropolis(loglik, log_prior, start, cov, m, rng):
    lchol = np.linalg.cholesky(cov)
    cur = np.array(start, dtype=np.float64)
    lp = loglik(cur) + log_prior(cur)
    out = np.empty((m, cur.size))
    acc = 0
    for t in range(m):
        prop = cur + lchol @ rng.standard_normal(cur.size)
        lpr = log_prior(prop)
        if np.isfinite(lpr):
            lq = loglik(prop) + lpr
            if math.log(rng.random()) < lq - lp:
                cur, lp = prop, lq
                acc += 1
        out[t] = cur
    return out, acc / m


@pytest.mark.parametrize("name", ["nn1d", "lf1d"])
def test_marginal_metropolis_matches_gibbs_posterior(hbm, name):
    wl = WORKLOADS[name](400)
    m = 30000
    _say(f"{name}: MWG chain vs random-walk Metropolis on the marginal likelihood, {m} steps each")
    s = hbm.Sampler(wl, max_cycles=m)
    s.run_cycles(m)
    tg = s.theta_trace()[m // 5:]
    o = oracle.Oracle(wl)
    cov = np.cov(tg.T) * (2.38 ** 2 / wl.p)
    rng = np.random.default_rng(9)
    ll = lambda th: float(s.marginal_loglik(th)[0])     # called only inside the prior's support
    tm, rate = _rw_metropolis(ll, o.log_prior, tg.mean(axis=0), cov, m, rng)
    tm = tm[m // 10:]
    _say(f"  marginal Metropolis acceptance {rate:.2f}")
    for j in range(wl.p):
        mg, sg = batch_means(tg[:, j], MOMENT_BATCHES)
        mm, sm = batch_means(tm[:, j], MOMENT_BATCHES)
        z = abs(mg - mm) / math.hypot(sg, sm)
        _say(f"  theta[{j}] gibbs {mg:.5f}±{sg:.5f} marginal {mm:.5f}±{sm:.5f} z={z:.2f}")
        assert z < 4.0
        # the two posterior spreads agree too
        assert 0.8 < np.std(tm[:, j]) / np.std(tg[:, j]) < 1.25
    s.close()


def test_argument_errors(hbm):
    wl3 = synth.normal_normal_3d(n=300)
    s3 = hbm.Sampler(wl3, max_cycles=4)
    with pytest.raises(hbm.HbmError, match="1-D latent"):
        s3.marginal_loglik([0.0, 0.0, 0.0])
    s3.close()
    wl = synth.gamma_lf_1d(n=300, seed=3, fth=389.75)
    s = hbm.Sampler(wl, max_cycles=4)
    with pytest.raises(hbm.HbmError, match="domain"):
        s.marginal_loglik([-1.0, wl.theta_true[1]])
    with pytest.raises(hbm.HbmError, match="finite"):
        s.marginal_loglik([math.nan, wl.theta_true[1]])
    # the context stays usable after a rejected call
    assert np.isfinite(s.marginal_loglik(wl.theta_true)[0])
    s.close()
