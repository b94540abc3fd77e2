"""Lockstep comparison of the GPU sampler with the FP64 oracle.

From one state (latents, RAM factors, theta, its factor, sweep count) both
sides take one RAM sweep with the same Philox streams; the oracle then
adopts the GPU's post-sweep latents and both take the theta step.  What is
compared, per object and per step:
  * log pi(X) and log pi(Y): |gpu - orc| <= rel * max(1, |orc|)  (rel = 1e-5
    for FP32 per-object arithmetic, 1e-12 for FP64);
  * accept/reject decisions: identical, except logged near-ties, where a
    mismatch is a near-tie only when the observed numeric error straddles
    the threshold, |ln u - Delta_orc| <= |Delta_gpu - Delta_orc|, and that
    error itself is within the tolerance above.  The same rule covers the
    decisions that the single-precision proposal point alone flips: the
    oracle's decision at the GPU's Y differs from its decision at its own
    Y_orc only where Y and Y_orc agree to the latent tolerance and ln u lies
    between the oracle's Delta at the two points.  Every near-tie is counted
    and the count is capped (max_near_ties);
  * the new latent (rejected: unchanged bit for bit; accepted: the
    proposal, equal up to the per-object precision) and the new RAM factor;
  * the theta step's log acceptance ratio, its decision (same near-tie
    rule) and the new theta and factor.
"""

from __future__ import annotations

import dataclasses

import numpy as np

import oracle


@dataclasses.dataclass
class StepReport:
    n: int
    max_rel_lpx: float
    max_rel_lpy: float
    near_ties: int               # all logged near-ties (value and proposal-point ones)
    decision_mismatch: int       # GPU decision != oracle decision at the GPU's own Y
    proposal_near_ties: int      # oracle decision at Y_gpu != at Y_orc
    max_chi_err: float
    max_chol_rel: float
    theta_delta_gpu: float
    theta_delta_orc: float
    theta_tol: float
    theta_near_tie: bool


def tolerances(precision: str):
    if precision == "f32":
        return dict(lp=1e-5, chi_ulps=8.0, chol=2e-5, theta_rel=1e-6)
    return dict(lp=1e-12, chi_ulps=64.0, chol=1e-11, theta_rel=1e-12)


def default_near_tie_cap(n: int) -> int:
    """Near-ties allowed in one sweep of n objects: a decision flips only when
    ln u falls within the per-object rounding (~1e-6 of log pi) of Delta, so
    a few per 10^5 objects at most."""
    return 3 + n // 20000


def _proposal_ulps(chi0, chol0, prec):
    """The rounding scale of Y = X + S U per component and object: the
    larger of |X| and the Box-Muller radius bound (sqrt(-2 ln 2^-24) = 5.77)
    times the row of S, in units of the per-object precision."""
    d = chi0.shape[0]
    rows = np.zeros_like(chi0)
    for r in range(d):
        for q in range(r + 1):
            rows[r] += np.abs(chol0[r * (r + 1) // 2 + q])
    size = np.maximum(np.abs(chi0), 5.77 * rows)
    return np.spacing(size.astype(np.float32 if prec == "f32" else np.float64)).astype(np.float64)


def lockstep_step(sampler, orc: "oracle.Oracle", prec: str, max_near_ties: int = None) -> StepReport:
    tol = tolerances(prec)
    chi0, chol0, acc0 = sampler.state()
    theta0, cth0, k0 = sampler.theta()
    tr = sampler.trace_sweep()                      # GPU sweep k0 + 1
    chi1, chol1, acc1 = sampler.state()

    st = oracle.State(chi0.copy(), chol0.copy(), acc0.copy(), theta0.copy(), cth0.copy(), k0)
    otr = orc.sweep(st, trace=True)                 # oracle sweep from the same state

    lpx_o, lnu_o, acc_o = otr[:, 0], otr[:, 2], otr[:, 3] > 0
    d = chi0.shape[0]
    lpx_g, lpy_g, acc_g, y_g = tr[0], tr[1], tr[2] > 0, tr[3:3 + d]
    # The GPU proposes Y in its own precision; both sides are compared at
    # that point (the oracle's exact-arithmetic proposal is checked against
    # it below, for the moves both sides accepted).
    lpy_o = orc.log_post(theta0, y_g)
    scale_x = np.maximum(1.0, np.abs(lpx_o))
    rel_x = np.abs(lpx_g - lpx_o) / scale_x
    fin_y = np.isfinite(lpy_o)
    rel_y = np.zeros_like(lpy_o)
    rel_y[fin_y] = np.abs(lpy_g[fin_y] - lpy_o[fin_y]) / np.maximum(1.0, np.abs(lpy_o[fin_y]))
    assert np.all(rel_x <= tol["lp"]), ("log pi(X)", rel_x.max(), int(np.argmax(rel_x)))
    assert np.all(rel_y <= tol["lp"]), ("log pi(Y)", rel_y.max(), int(np.argmax(rel_y)))
    # where the oracle's density at Y is zero the GPU must reject
    assert not np.any(acc_g & ~fin_y)

    delta_o = np.where(fin_y, lpy_o - lpx_o, -np.inf)
    acc_at_y = lnu_o < delta_o                       # the oracle's decision at the GPU's proposal
    mism = np.nonzero(acc_g != acc_at_y)[0]
    near = 0
    for i in mism:
        d_o = delta_o[i]
        d_g = lpy_g[i] - lpx_g[i]
        # the GPU's ln u is its own single-precision log of the same uniform
        err = abs(d_g - d_o) + (3e-7 * abs(lnu_o[i]) + 1e-7 if prec == "f32" else 1e-15)
        ok = abs(lnu_o[i] - d_o) <= err and err <= tol["lp"] * max(1.0, abs(lpx_o[i]), abs(lpy_o[i]))
        assert ok, ("decision mismatch that is not a near-tie", int(i), d_o, d_g, lnu_o[i])
        near += 1
    # Decisions the proposal point's rounding alone flipped: the oracle
    # decides differently at the GPU's Y than at its own exact-arithmetic
    # Y_orc.  Each must be a genuine straddle: Y and Y_orc within the latent
    # tolerance, and ln u between the oracle's Delta at the two points.
    ulp_all = _proposal_ulps(chi0, chol0, prec)
    flips = np.nonzero(acc_at_y != acc_o)[0]
    k_sweep = k0 + 1
    for i in flips:
        _, z = oracle.variates(orc.seed, [int(i), int(k_sweep), 0, 0])
        y_o = np.zeros(d)
        for r in range(d):
            y_o[r] = chi0[r, i] + sum(chol0[r * (r + 1) // 2 + q, i] * z[q] for q in range(r + 1))
        dy = np.abs(y_g[:, i] - y_o) / np.maximum(ulp_all[:, i], 1e-300)
        assert dy.max() <= tol["chi_ulps"], ("proposal near-tie with a distant proposal", int(i), dy.max())
        d_at_yo = otr[i, 1] - otr[i, 0] if np.isfinite(otr[i, 1]) else -np.inf
        d_at_yg = delta_o[i]
        gap = abs(d_at_yg - d_at_yo) if np.isfinite(d_at_yo) and np.isfinite(d_at_yg) else np.inf
        assert abs(lnu_o[i] - d_at_yo) <= gap + 1e-15 * max(1.0, abs(lnu_o[i])), \
            ("proposal flip that does not straddle ln u", int(i), d_at_yo, d_at_yg, lnu_o[i])
    near_prop = int(len(flips))
    near += near_prop
    cap = default_near_tie_cap(sampler.n) if max_near_ties is None else max_near_ties
    assert near <= cap, ("near-ties above the cap", near, cap)

    same = acc_g == acc_o
    # rejected moves keep the latent bit for bit
    rej = same & ~acc_o
    assert np.array_equal(chi1[:, rej], chi0[:, rej])
    # accepted moves land on the proposal Y = X + S U.  Its error is set by
    # the operands, not by Y (a latent near zero can cancel): the rounding of
    # X and the single-precision normals' absolute error, which scales with
    # the Box-Muller radius (at most sqrt(-2 ln 2^-24) = 5.77) times the row
    # of S
    accd = same & acc_o
    ulp = ulp_all[:, accd]
    err = np.abs(chi1[:, accd] - st.chi[:, accd])
    chi_err = float((err / np.maximum(ulp, 1e-300)).max()) if err.size else 0.0
    assert chi_err <= tol["chi_ulps"], ("latent", chi_err)
    crel = np.abs(chol1[:, same] - st.chol[:, same]) / np.maximum(np.abs(st.chol[:, same]), 1e-30)
    # off-diagonal factor entries can be tiny; compare them relative to the diagonal scale
    if d > 1:
        diag_idx = [r * (r + 1) // 2 + r for r in range(d)]
        dscale = np.max(np.abs(st.chol[diag_idx][:, same]), axis=0)
        crel = np.abs(chol1[:, same] - st.chol[:, same]) / np.maximum(dscale, 1e-30)
    # The factor adapts on alpha = min(1, e^Delta): with the two sides' Delta
    # apart by dD, |d alpha| <= alpha_max dD (alpha is 1-Lipschitz in Delta
    # below 0, scaled by its value), and eq 2.6 moves the factor by at most
    # eta |d alpha| / (2 (1 + c)) < eta |d alpha| relative in 1-D (1 + c >=
    # 1 - eta alpha* > 0.7); allow twice that in more dimensions, where the
    # rank-1 term is measured against the largest diagonal entry.  The
    # constant tol["chol"] covers the factor's own single-precision rounding.
    d_gg = np.where(np.isfinite(lpy_g), lpy_g - lpx_g, -np.inf)
    d_oo = np.where(np.isfinite(otr[:, 1]), otr[:, 1] - otr[:, 0], -np.inf)
    both = np.isfinite(d_gg) & np.isfinite(d_oo)
    a_max = np.exp(np.minimum(0.0, np.maximum(d_gg, d_oo)))
    dalpha = np.where(both, np.minimum(1.0, a_max * np.abs(np.where(both, d_gg - d_oo, 0.0))), a_max)
    eta = (k0 + 2) ** (-getattr(orc, "gamma", 2.0 / 3.0))
    bound = tol["chol"] + (1.0 if d == 1 else 2.0) * eta * dalpha[same]
    worst = crel - bound[None, :] if crel.size else np.zeros(1)
    chol_rel = float(crel.max()) if crel.size else 0.0
    assert np.all(worst <= 0.0), ("RAM factor", chol_rel, float(worst.max()), int(np.nonzero(same)[0][
        np.argmax(worst.max(axis=0))]))
    assert np.array_equal(acc1[same], st.acc[same])

    # theta step: the oracle takes the GPU's latents (lockstep)
    st.chi = chi1.copy()
    st.chol = chol1.copy()
    st.acc = acc1.copy()
    prop = orc.theta_proposal(st, k=k0 + 1)
    scale = float(np.sum(np.abs(orc.pop_terms(prop, chi1) - orc.pop_terms(theta0, chi1)))) \
        if np.isfinite(orc.log_prior(prop)) else 0.0
    info = orc.theta_step(st)
    acc_th_g = sampler.theta_step()
    stats = sampler.stats()
    theta1, cth1, _ = sampler.theta()
    d_g, d_o = stats["delta"], info["delta"]
    n_sub = getattr(orc, "theta_substeps", 1)
    if n_sub > 1:
        # K steps on theta: the same number accepted, the same theta, the
        # last step's log ratio within the tolerance (a near-tie inside the
        # K steps would show as a different count)
        has_sel = orc.wl.model in (2, 3, 5)
        pl, tb = info["prop_last"], info["theta_before_last"]
        scale, mag = 0.0, 0.0
        if np.isfinite(orc.log_prior(pl)):
            lp_p, lp_c = orc.pop_terms(pl, chi1), orc.pop_terms(tb, chi1)
            scale = float(np.sum(np.abs(lp_p - lp_c)))
            mag = float(np.sum(np.abs(lp_p)) + np.sum(np.abs(lp_c)))
        # the statistics give Delta as a difference of N-term sums: in FP64 it
        # carries rounding of the order of an ulp of the terms' magnitudes, not
        # of their differences (in FP32 the per-object rounding dominates)
        theta_tol = tol["theta_rel"] * max(1.0, scale) + (1e-12 * sampler.n if has_sel else 0.0) + \
            (1e-14 * mag if prec == "f64" else 0.0)
        assert int(acc_th_g) == info["n_accepted"], ("theta steps accepted", int(acc_th_g), info["n_accepted"])
        if np.isfinite(d_o):
            assert abs(d_g - d_o) <= theta_tol, ("theta delta", d_g, d_o, theta_tol)
        # later proposals start from a factor adapted on alpha = min(1, e^Delta):
        # each step moves the factor by at most |d Delta| relative, and a
        # proposal by that times the step S z (a few diagonal scales)
        dd = abs(d_g - d_o) if np.isfinite(d_o) else 0.0
        rt = 1e-8 + 10.0 * n_sub * dd
        scale_th = float(np.abs(np.diag(st.chol_theta)).max())
        np.testing.assert_allclose(theta1, st.theta, rtol=rt, atol=rt * scale_th)
        np.testing.assert_allclose(cth1, st.chol_theta, rtol=rt, atol=rt * scale_th)
        return StepReport(sampler.n, float(rel_x.max()), float(rel_y.max()), near, len(mism), near_prop, chi_err,
                          chol_rel, d_g, d_o, theta_tol, False)
    # FP64 selection normalisers of the two sides agree to ~1e-13 relative
    has_sel = orc.wl.model in (2, 3, 5)
    theta_tol = tol["theta_rel"] * max(1.0, scale) + (1e-12 * sampler.n if has_sel else 0.0)
    near_theta = False
    if np.isfinite(d_o):
        assert abs(d_g - d_o) <= theta_tol, ("theta delta", d_g, d_o, theta_tol)
    else:
        assert not np.isfinite(d_g)
    if acc_th_g != info["accepted"]:
        assert abs(info["ln_u"] - d_o) <= abs(d_g - d_o) <= theta_tol, ("theta decision", d_g, d_o, info["ln_u"])
        near_theta = True
    else:
        np.testing.assert_allclose(theta1, st.theta, rtol=1e-12, atol=1e-12)
        # S_theta adapts on alpha = min(1, e^Delta); |d alpha| <= |d Delta|, and the
        # factor moves by at most eta |d alpha| relative, so the two factors may
        # differ by the Delta discrepancy of the per-object precision
        rt = 1e-9 + 2.0 * (abs(d_g - d_o) if np.isfinite(d_o) else 0.0)
        scale_th = float(np.abs(np.diag(st.chol_theta)).max())
        np.testing.assert_allclose(cth1, st.chol_theta, rtol=rt, atol=rt * scale_th)
    return StepReport(sampler.n, float(rel_x.max()), float(rel_y.max()), near, len(mism), near_prop, chi_err,
                      chol_rel, d_g, d_o, theta_tol, near_theta)
