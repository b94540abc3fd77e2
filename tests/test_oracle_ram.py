"""Pins for the oracle's robust adaptive Metropolis step (Sec. 2.2, eq 2.6).

  * One-step algebra, recomputed independently with numpy from the same
    random draws: Y = X + S U, the accept rule ln u < log pi(Y) - log pi(X),
    and S_n S_n^T = S (I + eta (alpha - alpha*) U U^T / |U|^2) S^T with S_n
    equal to numpy's Cholesky factor of that matrix (lower, positive
    diagonal); in 1-D this is S_n = S sqrt(1 + eta (alpha - alpha*)).
  * The determinant identity ln det S_n - ln det S = 1/2 ln(1 + eta (alpha - alpha*)).
  * Long-run invariants on a Gaussian target: mean acceptance -> alpha*,
    and the proposal scale -> s* = 2 sigma / tan(alpha* pi / 2), which
    follows from the closed-form acceptance (2/pi) arctan(2 sigma / s) of a
    Gaussian random walk on N(0, sigma^2).
  * With theta fixed the latent chains sample the closed-form conditional
    N(m_i, v_i) of the normal-normal model.
"""
import math

import numpy as np
import pytest

import synth


def _packed_to_dense(chol, i, d):
    s = np.zeros((d, d))
    e = 0
    for r in range(d):
        for c in range(r + 1):
            s[r, c] = chol[e, i]
            e += 1
    return s


@pytest.mark.parametrize("wl_fn", [lambda: synth.normal_normal_3d(n=200), lambda: synth.gamma_lf_3d(n=200, seed=31),
                                   lambda: synth.gamma_lf_1d(n=200, seed=32), lambda: synth.normal_normal_1d(n=200)])
def test_one_ram_step_algebra(oracle_lib, wl_fn):
    wl = wl_fn()
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    o.run(st, 150)                    # let the factors adapt away from S = I
    d, n, k = wl.d, wl.n, st.k + 1
    before = st.copy()
    tr = o.sweep(st, trace=True)
    eta = (k + 1) ** (-2.0 / 3.0)
    n_acc = 0
    for i in range(n):
        u, z = oracle_lib.variates(wl.seed, [i, k, 0, 0])
        uvec = z[:d]
        s_old = _packed_to_dense(before.chol, i, d)
        x = before.chi[:, i]
        y = x + s_old @ uvec
        lm_x, lp_x = o.log_terms(i, x, before.theta)
        lm_y, lp_y = o.log_terms(i, y, before.theta)
        assert tr[i, 0] == pytest.approx(lm_x + lp_x, rel=1e-14, abs=1e-12)
        if np.isfinite(lm_y + lp_y):
            # y is recomputed here with numpy's summation order: last-bit differences
            assert tr[i, 1] == pytest.approx(lm_y + lp_y, rel=1e-11, abs=1e-12)
        delta = (lm_y + lp_y) - (lm_x + lp_x) if np.isfinite(lm_y + lp_y) else -np.inf
        acc = math.log(u[4]) < delta
        if abs(math.log(u[4]) - delta) > 1e-9:
            assert bool(tr[i, 3]) == acc
        acc = bool(tr[i, 3])
        assert tr[i, 4] == pytest.approx(min(1.0, math.exp(delta)) if delta > -np.inf else 0.0, rel=1e-10)
        np.testing.assert_allclose(st.chi[:, i], y if acc else x, rtol=1e-14, atol=1e-14)
        n_acc += acc
        c = eta * (tr[i, 4] - wl.alpha_star)
        s_new = _packed_to_dense(st.chol, i, d)
        if not uvec.dot(uvec) > 0.0:
            # U = 0: the limit of eq 2.6 in 1-D, no change in more dimensions
            want = s_old * math.sqrt(1 + c) if d == 1 else s_old
            np.testing.assert_allclose(s_new, want, rtol=1e-14)
            continue
        target = s_old @ (np.eye(d) + c * np.outer(uvec, uvec) / uvec.dot(uvec)) @ s_old.T
        np.testing.assert_allclose(s_new, np.linalg.cholesky(target), rtol=1e-12, atol=1e-14)
        assert np.all(np.diag(s_new) > 0) and np.allclose(np.triu(s_new, 1), 0)
        # determinant identity of eq (2.6)
        ld = np.sum(np.log(np.diag(s_new))) - np.sum(np.log(np.diag(s_old)))
        assert ld == pytest.approx(0.5 * math.log1p(c), rel=1e-11, abs=1e-14)
        if d == 1:
            assert s_new[0, 0] == pytest.approx(s_old[0, 0] * math.sqrt(1 + c), rel=1e-14)
    assert np.array_equal(st.acc - before.acc, (tr[:, 3] > 0).astype(np.uint32))
    assert 0 < n_acc < n


def test_zero_proposal_direction_in_1d(oracle_lib):
    """The 24-bit variate map reaches u0 = 1 (field 0xFFFFFF), where the
    Box-Muller radius and so U are exactly 0.  Key 1 (the 300,000-object
    luminosity-function catalog), object 153325, sweep 63 is such a draw.
    There Y = X, so Delta = 0 and alpha = 1, and eq 2.6 in one dimension
    gives the limit of chol(S (1 + c U^2 / U^2) S) as U -> 0: S sqrt(1 + c)
    with c = eta_63 (1 - alpha*).  The limit is taken here from the matrix
    definition itself at a tiny nonzero U (numpy's Cholesky), not from the
    oracle's formula."""
    i, k = 153325, 63
    u, z = oracle_lib.variates(1, [i, k, 0, 0])
    assert u[0] == 1.0 and z[0] == 0.0
    wl = synth.gamma_lf_1d(n=i + 1, seed=1, fth=389.75)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state(s0=0.3)
    st.k = k - 1
    x0 = st.chi[0, i]
    tr = o.sweep(st, trace=True)
    assert st.k == k
    assert tr[i, 1] == tr[i, 0] and tr[i, 4] == 1.0          # Y = X: Delta = 0, alpha = 1
    assert st.chi[0, i] == x0
    c = (k + 1) ** (-2.0 / 3.0) * (1.0 - wl.alpha_star)
    tiny = 1e-150
    limit = np.linalg.cholesky(np.array([[0.3 * (1.0 + c * tiny * tiny / (tiny * tiny)) * 0.3]]))[0, 0]
    assert st.chol[0, i] == pytest.approx(limit, rel=1e-15)
    assert st.chol[0, i] == pytest.approx(0.3 * 1.01734, rel=1e-5)    # the 1.7 % step a skip would miss
    # every other object of the sweep still follows the matrix definition
    for j in (0, 1, i - 1):
        _, zj = oracle_lib.variates(1, [j, k, 0, 0])
        assert zj[0] != 0.0
        cj = (k + 1) ** (-2.0 / 3.0) * (tr[j, 4] - wl.alpha_star)
        assert st.chol[0, j] == pytest.approx(0.3 * math.sqrt(1.0 + cj), rel=1e-14)


def _nn1_fixed_theta_run(oracle_lib, n_sweeps, thin):
    wl = synth.normal_normal_1d(n=1000, seed=0)
    o = oracle_lib.Oracle(wl)
    st = o.initial_state()
    _, ct = o.run(st, n_sweeps, thin=thin, fix_theta=True, chi_trace=True)
    y, sig = wl.data
    v = 1.0 / (1.0 / sig**2 + 1.0)        # theta fixed at the truth: mu = 0, tau = 1
    m = v * (y / sig**2)
    return wl, st, ct[:, 0, :], m, v


def test_ram_acceptance_and_scale_fixed_points(oracle_lib):
    n_sweeps = 20000
    wl, st, ct, m, v = _nn1_fixed_theta_run(oracle_lib, n_sweeps, thin=20)
    s_star = 2.0 / math.tan(wl.alpha_star * math.pi / 2)          # 2.4176 at alpha* = 0.44
    assert s_star == pytest.approx(2.4176, abs=1e-4)
    ratio = np.log(st.chol[0] / np.sqrt(v))
    assert np.mean(ratio) == pytest.approx(math.log(s_star), abs=0.01)
    assert np.all(np.abs(ratio - math.log(s_star)) < 0.25)
    assert st.acc.mean() / n_sweeps == pytest.approx(wl.alpha_star, abs=0.01)


def test_latent_chains_sample_the_conditional(oracle_lib):
    from conftest import batch_means
    wl, st, ct, m, v = _nn1_fixed_theta_run(oracle_lib, 30000, thin=10)
    keep = ct[ct.shape[0] // 5:]
    mean, se = batch_means(keep)
    t = (mean - m) / se
    assert abs(np.mean(t)) < 4.0 / math.sqrt(len(t))      # pooled over 1000 independent chains
    assert 0.8 < np.std(t) < 1.25
    var_ratio = keep.var(axis=0) / v
    assert np.mean(var_ratio) == pytest.approx(1.0, abs=0.02)


def test_resume_is_bit_identical(oracle_lib):
    wl = synth.gamma_lf_1d(n=500, seed=33)
    o = oracle_lib.Oracle(wl)
    a = o.initial_state()
    b = o.initial_state()
    ta, _ = o.run(a, 30)
    tb1, _ = o.run(b, 11)
    tb2, _ = o.run(b, 19)
    assert np.array_equal(ta, np.vstack([tb1, tb2]))
    assert np.array_equal(a.chi, b.chi) and np.array_equal(a.chol, b.chol)
    assert np.array_equal(a.acc, b.acc) and np.array_equal(a.theta, b.theta)
    assert np.array_equal(a.chol_theta, b.chol_theta)
