"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

FP64 models (normal-normal, 1-D and the paper's 3-D instance): whole chains
must coincide with the oracle's (identical decisions; values to ~1e-12).
FP32 models (luminosity function, 1-D and 3-D): lockstep, one sweep and
one theta step at a time from a shared state (tests/lockstep.py), at sizes
that span several 256-object tiles and a ragged tail, and at the full
300,000-object catalog in the launch configuration the bench uses.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import INDEPENDENT_SEED, assert_moments_agree, moment_scores
from lockstep import lockstep_step

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


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


def test_nn1d_chain_identical_to_oracle(hbm):
    _say("nn1d chain: N=1000, 2000 cycles, plain ram_sweep + theta_step")
    wl = synth.normal_normal_1d(n=1000, seed=0)
    s = hbm.Sampler(wl, max_cycles=2000)
    for _ in range(2000):
        s.ram_sweep(1)
        s.theta_step()
    tg = s.theta_trace()
    chi_g, chol_g, acc_g = s.state()
    o = oracle.Oracle(wl)
    st = o.initial_state()
    to, _ = o.run(st, 2000)
    np.testing.assert_allclose(tg, to, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(chi_g, st.chi, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(chol_g, st.chol, rtol=1e-10)
    assert np.array_equal(acc_g, st.acc)


def test_nn1d_fused_graph_equals_plain(hbm):
    _say("nn1d: run_cycles (graph, fused theta step) vs ram_sweep + theta_step, bitwise")
    wl = synth.normal_normal_1d(n=1000, seed=0)
    a = hbm.Sampler(wl, max_cycles=300)
    for _ in range(300):
        a.ram_sweep(1)
        a.theta_step()
    b = hbm.Sampler(wl, max_cycles=300)
    b.run_cycles(300, use_graph=True)
    c = hbm.Sampler(wl, max_cycles=300)
    c.run_cycles(300, use_graph=False)
    for other in (b, c):
        assert np.array_equal(a.theta_trace(), other.theta_trace())
        sa, so = a.state(), other.state()
        for x, y in zip(sa, so):
            assert np.array_equal(x, y)


def test_graph_replays_cover_any_length(hbm):
    """run_cycles with graphs replays a 32-cycle graph and one graph of the
    remainder, for any length, with the chain of plain launches."""
    wl = synth.gamma_lf_1d(n=2000, seed=59, fth=389.75)
    a = hbm.Sampler(wl, max_cycles=100)
    a.set_cycle_mode(hbm.HBM_CYCLES_GRAPH)      # graphs, not the persistent launch
    b = hbm.Sampler(wl, max_cycles=100)
    a.prepare_cycles(20)
    lc = a.launch_counts()
    assert lc["graph_captures"] == 1 and lc["graph_replays"] == 0
    a.run_cycles(20)
    lc = a.launch_counts()
    assert (lc["graph_replays"], lc["replayed_cycles"], lc["plain_cycles"], lc["graph_captures"]) == (1, 20, 0, 1)
    a.run_cycles(75)                 # 2 x 32 + a new remainder graph of 11
    lc = a.launch_counts()
    assert (lc["graph_replays"], lc["replayed_cycles"], lc["graph_captures"]) == (4, 95, 3)
    b.run_cycles(95, use_graph=False)
    assert b.launch_counts()["plain_cycles"] == 95
    assert np.array_equal(a.theta_trace(), b.theta_trace())
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_nn3d_papers_instance_chain_identical(hbm):
    _say("nn3d (paper Sec. 3 instance): N=777, 400 cycles")
    wl = synth.normal_normal_3d(n=777, seed=5)
    s = hbm.Sampler(wl, max_cycles=400)
    s.run_cycles(400, use_graph=True)
    o = oracle.Oracle(wl)
    st = o.initial_state()
    to, _ = o.run(st, 400)
    np.testing.assert_allclose(s.theta_trace(), to, rtol=1e-9, atol=1e-9)
    chi_g, chol_g, acc_g = s.state()
    np.testing.assert_allclose(chi_g, st.chi, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(chol_g, st.chol, rtol=1e-8, atol=1e-10)
    assert np.array_equal(acc_g, st.acc)


@pytest.mark.parametrize("n", [3001, 257])
def test_lf1d_lockstep(hbm, n):
    _say(f"lf1d lockstep: N={n}")
    wl = synth.gamma_lf_1d(n=n, seed=51, fth=389.75)
    s = hbm.Sampler(wl, max_cycles=200)
    o = oracle.Oracle(wl)
    worst = 0.0
    for step in range(40):
        r = lockstep_step(s, o, "f32")
        worst = max(worst, r.max_rel_lpx, r.max_rel_lpy)
        if step % 10 == 0:
            _say(f"  step {step}: max rel lp err {worst:.2e} near-ties {r.near_ties} dtheta {r.theta_delta_gpu - r.theta_delta_orc:.2e}")


def test_lf3d_lockstep(hbm):
    _say("lf3d lockstep: N=3001")
    wl = synth.gamma_lf_3d(n=3001, seed=52, fth=389.75)
    s = hbm.Sampler(wl, max_cycles=200)
    o = oracle.Oracle(wl)
    for step in range(30):
        r = lockstep_step(s, o, "f32")
        if step % 10 == 0:
            _say(f"  step {step}: lp err {max(r.max_rel_lpx, r.max_rel_lpy):.2e} chol {r.max_chol_rel:.2e}")


def test_lf1d_lockstep_through_zero_proposal_direction(hbm):
    """Sweep 63 of the 300,000-object catalog (key 1) draws u0 = 1 for
    object 153325: the Box-Muller radius and U are exactly 0, Y = X, and the
    1-D RAM step scales the factor by sqrt(1 + eta_63 (1 - alpha*)) (eq 2.6
    in one dimension).  The whole sweep runs in lockstep with the oracle from
    a state at sweep 62, so that object's factor is compared too."""
    _say("lf1d full catalog N=300000: lockstep of sweep 63 (object 153325 has U = 0)")
    wl = synth.gamma_lf_1d()
    assert wl.seed == 1 and wl.n > 153325
    s = hbm.Sampler(wl, max_cycles=8)
    th, cth, _ = s.theta()
    s.set_theta(th, cth, 62)
    chi0, chol0, _ = s.state()
    o = oracle.Oracle(wl)
    r = lockstep_step(s, o, "f32")
    _say(f"  lp err {max(r.max_rel_lpx, r.max_rel_lpy):.2e} chol {r.max_chol_rel:.2e} near-ties {r.near_ties}")
    chi1, chol1, _ = s.state()
    i = 153325
    assert chi1[0, i] == chi0[0, i]
    want = chol0[0, i] * math.sqrt(1.0 + 64.0 ** (-2.0 / 3.0) * (1.0 - wl.alpha_star))
    assert abs(chol1[0, i] - want) <= 2e-6 * want, (chol1[0, i], want)
    s.close()


def test_lf1d_full_catalog_lockstep_after_graph_cycles(hbm):
    _say("lf1d full catalog N=300000: 200 graph cycles, then 3 lockstep steps")
    wl = synth.gamma_lf_1d()
    s = hbm.Sampler(wl, max_cycles=400)
    s.run_cycles(200, use_graph=True)
    o = oracle.Oracle(wl)
    for _ in range(3):
        r = lockstep_step(s, o, "f32")
        _say(f"  lp err {max(r.max_rel_lpx, r.max_rel_lpy):.2e} near-ties {r.near_ties}")
    th = s.theta_trace()
    assert np.all(np.isfinite(th))


def test_lf3d_full_catalog_lockstep_after_graph_cycles(hbm):
    """The 3-D colour catalog at its full size (N = 10^6) in the launch shape
    the bench picks: autotuned burn-in and graph-replayed cycles, then whole
    sweeps in lockstep with the oracle (every object checked)."""
    _say("lf3d full catalog N=1000000: autotune + 100 graph cycles, then 2 lockstep steps")
    wl = synth.gamma_lf_3d()
    s = hbm.Sampler(wl, max_cycles=hbm.autotune_cycles(16) + 110)
    pick, us = s.autotune(16)
    _say(f"  choice {pick}; us/cycle {dict(zip(hbm.tune_labels(), np.round(us, 2)))}")
    s.run_cycles(100, use_graph=True)
    o = oracle.Oracle(wl)
    for _ in range(2):
        r = lockstep_step(s, o, "f32")
        _say(f"  lp err {max(r.max_rel_lpx, r.max_rel_lpy):.2e} chol {r.max_chol_rel:.2e} near-ties {r.near_ties}")
    assert np.all(np.isfinite(s.theta_trace()))
    s.close()


@pytest.mark.parametrize("make", [lambda: synth.normal_normal_1d(n=1000),
                                  lambda: synth.gamma_lf_1d(n=5000, seed=53, fth=389.75),
                                  lambda: synth.gamma_lf_3d(n=2000, seed=54, fth=389.75),
                                  lambda: synth.normal_normal_3d(n=500)])
def test_pop_loglik_matches_oracle(hbm, make):
    wl = make()
    _say(f"pop_loglik {wl.name} N={wl.n}")
    s = hbm.Sampler(wl, max_cycles=50)
    s.run_cycles(20)
    chi, _, _ = s.state()
    o = oracle.Oracle(wl)
    rng = np.random.default_rng(9)
    for _ in range(4):
        th = wl.theta_true + 0.02 * rng.standard_normal(wl.p) * np.abs(np.diag(wl.theta_chol0)) / 0.05
        if not np.isfinite(o.log_prior(th)):
            continue
        got = s.pop_loglik(th)
        ref = o.pop_loglik(th, chi)
        scale = np.sum(np.abs(o.pop_terms(th, chi)))
        rel = 1e-6 if wl.precision == "f32" else 1e-13
        assert abs(got - ref) <= rel * scale + 1e-12 * wl.n, (got, ref, scale)


def test_determinism_and_stats(hbm):
    _say("determinism: two contexts, same seed, fused graph path")
    wl = synth.gamma_lf_1d(n=20000, seed=55, fth=389.75)
    a = hbm.Sampler(wl, max_cycles=100)
    b = hbm.Sampler(wl, max_cycles=100)
    a.run_cycles(100)
    b.run_cycles(100)
    assert np.array_equal(a.theta_trace(), b.theta_trace())
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    st = a.stats()
    assert 0 <= st["n_acc"] <= wl.n and np.isfinite(st["sum_lf"])


def test_error_paths(hbm):
    wl = synth.gamma_lf_1d(n=1000, seed=56, fth=389.75)
    bad = synth.gamma_lf_1d(n=1000, seed=56, fth=389.75)
    bad.theta0 = np.array([0.5, bad.theta0[1]])          # beta outside (-1, 0)
    with pytest.raises(hbm.HbmError) as e:
        hbm.Sampler(bad)
    assert e.value.status == hbm.HBM_EDOMAIN
    s = hbm.Sampler(wl, max_cycles=2)
    with pytest.raises(hbm.HbmError) as e:
        s.theta_step()                                     # no sweep yet
    assert e.value.status == hbm.HBM_ESTATE
    s.run_cycles(2)
    with pytest.raises(hbm.HbmError) as e:
        s.run_cycles(1)                                    # trace full
    assert e.value.status == hbm.HBM_ENOSPACE
    # the context still works after validation errors
    assert np.isfinite(s.pop_loglik(wl.theta0))


def test_snapshots(hbm):
    wl = synth.normal_normal_1d(n=600)
    s = hbm.Sampler(wl, max_cycles=100, thin=10)
    s.run_cycles(100)
    snaps = s.chi_snapshots(0, 10)
    o = oracle.Oracle(wl)
    st = o.initial_state()
    _, ct = o.run(st, 100, thin=10, chi_trace=True)
    np.testing.assert_allclose(snaps, ct, rtol=1e-10, atol=1e-10)


def test_lf1d_free_run_posterior_moments(hbm):
    _say("lf1d free run: posterior theta moments vs oracle within MCSE")
    wl = synth.gamma_lf_1d(n=400, seed=57, fth=389.75)
    m = 30000
    s = hbm.Sampler(wl, max_cycles=m)
    s.run_cycles(m)
    tg = s.theta_trace()[m // 5:]
    # an independent oracle chain: its own Philox key, so the two chains'
    # batch-means errors add as the combined standard error assumes
    o = oracle.Oracle(wl, seed=INDEPENDENT_SEED)
    st = o.initial_state()
    to, _ = o.run(st, m)
    to = to[m // 5:]
    scores = moment_scores(tg, to)
    for j, (z, zv, mg, sg, mo, so) in enumerate(scores):
        _say(f"  theta[{j}] gpu {mg:.5f}±{sg:.5f} oracle {mo:.5f}±{so:.5f} z={z:.2f}; variance z={zv:.2f}")
    _say(f"  rms z over the means and variances {assert_moments_agree(scores):.2f}")


def test_lf3d_free_run_posterior_moments(hbm):
    """The 3-D colour model (p = 5): posterior means and variances of every
    theta component from a free GPU run against an independent FP64 oracle
    chain, within 2 combined batch-means MCSE (pooled over the ten
    moments).  The colour parameters mix slowly (integrated autocorrelation
    times of 730-960 cycles at N = 300, measured on the oracle), so both
    chains run 250,000 cycles and the standard errors use 20 batches of
    10,000 draws, about ten autocorrelation times each."""
    _say("lf3d free run: posterior theta moments (5 components) vs oracle within 2 MCSE")
    wl = synth.gamma_lf_3d(n=300, seed=58, fth=389.75)
    m = 250000
    s = hbm.Sampler(wl, max_cycles=m)
    s.run_cycles(m)
    tg = s.theta_trace()[m // 5:]
    s.close()
    # an independent oracle chain: its own Philox key, so the two chains'
    # batch-means errors add as the combined standard error assumes
    o = oracle.Oracle(wl, seed=INDEPENDENT_SEED)
    st = o.initial_state()
    to, _ = o.run(st, m)
    to = to[m // 5:]
    assert np.all(np.isfinite(tg))
    scores = moment_scores(tg, to, n_batches=20)
    for j, (z, zv, mg, sg, mo, so) in enumerate(scores):
        _say(f"  theta[{j}] gpu {mg:.5f}±{sg:.5f} oracle {mo:.5f}±{so:.5f} z={z:.2f}; variance z={zv:.2f}")
    _say(f"  rms z over the means and variances {assert_moments_agree(scores):.2f}")


@pytest.mark.parametrize("n", [1, 2])
def test_tiny_catalogs(hbm, n):
    """Degenerate sizes: one and two objects (one partial tile, 255 or 254
    idle lanes).  The normal-normal chain equals the oracle's; the LF chain
    runs in lockstep with it; every issue mode gives the same chain."""
    _say(f"tiny catalogs: N={n}")
    wl = synth.normal_normal_1d(n=n, seed=62)
    s = hbm.Sampler(wl, max_cycles=100)
    s.run_cycles(100)
    o = oracle.Oracle(wl)
    to, _ = o.run(o.initial_state(), 100)
    np.testing.assert_allclose(s.theta_trace(), to, rtol=1e-9, atol=1e-9)
    lf = synth.gamma_lf_1d(n=n, seed=61, fth=389.75)
    a = hbm.Sampler(lf, max_cycles=60)
    ol = oracle.Oracle(lf)
    for _ in range(10):
        lockstep_step(a, ol, "f32")
    runs = []
    for mode in (hbm.HBM_CYCLES_GRAPH, hbm.HBM_CYCLES_FUSED, hbm.HBM_CYCLES_AUTO):
        b = hbm.Sampler(lf, max_cycles=70)
        b.set_cycle_mode(mode)
        b.run_cycles(70)
        runs.append((b.theta_trace(), b.state()))
        b.close()
    for tr, st in runs[1:]:
        assert np.array_equal(tr, runs[0][0])
        for x, y in zip(st, runs[0][1]):
            assert np.array_equal(x, y)
