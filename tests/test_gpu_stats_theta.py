"""GPU parity of the sufficient-statistic theta path.

For exponential-family populations the sweep reduces a few per-object
statistics at the new latents (gamma law: sum (chi - ln L*), sum e^(chi -
ln L*); normal: sum (chi - mu), sum (chi - mu)^2; the colour regression adds
its residual moments), and the epilogue takes K Metropolis steps on theta
from them, every later proposal's selection normaliser summed on the spot.
The oracle takes the same K steps from the full N-term sums (the generic
path is the statistics' oracle).  Checks:

* lockstep sweeps and K-step theta updates against the oracle (K = 1 and 4)
  for the gamma LF (1-D and colour 3-D) and normal-normal (1-D and 3-D)
  models: same number of steps accepted, same theta, the last log ratio
  within the tolerance of the per-object precision;
* with K = 1 the statistics path makes the Gibbs sampler's own chain: its
  theta trace equals the generic path's;
* graph-replayed cycles equal plain sweep + theta-step calls, a batch equals
  each catalog alone, bit for bit;
* posterior moments with K = 4 agree with the generic sampler's;
* argument errors (BB1 has no sufficient statistics; modes cannot mix).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import MOMENT_BATCHES, batch_means
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


CASES = {
    "lf1d": (lambda: synth.gamma_lf_1d(n=3001, seed=81, fth=389.75), "f32"),
    "nn1d": (lambda: synth.normal_normal_1d(n=2000, seed=82), "f64"),
    "lf3d": (lambda: synth.gamma_lf_3d(n=1500, seed=83), "f32"),
    "nn3d": (lambda: synth.normal_normal_3d(n=1000, seed=84), "f64"),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("K", [1, 4])
def test_lockstep_with_oracle(hbm, name, K):
    gen, prec = CASES[name]
    wl = gen()
    _say(f"stats theta lockstep {name} K={K} N={wl.n}")
    s = hbm.Sampler(wl, max_cycles=100, theta_substeps=K)
    o = oracle.Oracle(wl, theta_substeps=K)
    for step in range(25):
        r = lockstep_step(s, o, prec)
        if step % 8 == 0:
            _say(f"  step {step}: theta delta gpu {r.theta_delta_gpu:.6e} orc {r.theta_delta_orc:.6e} "
                 f"tol {r.theta_tol:.1e}")
    s.close()


@pytest.mark.parametrize("name", ["lf1d", "nn3d"])
def test_one_substep_is_the_generic_chain(hbm, name):
    wl = CASES[name][0]()
    m = 200
    a = hbm.Sampler(wl, max_cycles=m)
    b = hbm.Sampler(wl, max_cycles=m, theta_substeps=1)
    a.run_cycles(m)
    b.run_cycles(m)
    ta, tb = a.theta_trace(), b.theta_trace()
    moved_a = np.any(np.diff(ta, axis=0) != 0, axis=1)
    moved_b = np.any(np.diff(tb, axis=0) != 0, axis=1)
    _say(f"  {name}: {int(moved_a.sum())} theta moves in {m} cycles; max |dtheta| {np.max(np.abs(ta - tb)):.2e}")
    assert np.array_equal(moved_a, moved_b)
    np.testing.assert_allclose(ta, tb, rtol=1e-6, atol=1e-6)
    a.close()
    b.close()


def test_graph_and_plain_cycles_agree(hbm):
    wl = synth.gamma_lf_1d(n=5000, seed=85, fth=389.75)
    g = hbm.Sampler(wl, max_cycles=80, theta_substeps=3)
    p = hbm.Sampler(wl, max_cycles=80, theta_substeps=3)
    g.run_cycles(80, use_graph=True)
    for _ in range(80):
        p.ram_sweep()
        p.theta_step()
    assert np.array_equal(g.theta_trace(), p.theta_trace())
    assert np.array_equal(g.state()[0], p.state()[0])
    g.close()
    p.close()


def test_batch_equals_alone(hbm):
    wls = [synth.gamma_lf_1d(n=n, seed=86 + j, fth=389.75) for j, n in enumerate((700, 2600, 300))]
    b = hbm.Batch(wls, max_cycles=60, theta_substeps=2)
    b.run_cycles(60)
    for j, w in enumerate(wls):
        s = hbm.Sampler(w, max_cycles=60, theta_substeps=2)
        s.run_cycles(60)
        assert np.array_equal(b.theta_trace(j), s.theta_trace()), j
        assert np.array_equal(b.latents(j), s.state()[0]), j
        s.close()
    b.close()


def test_posterior_moments_match_the_generic_sampler(hbm):
    wl = synth.gamma_lf_1d(n=400, seed=87, fth=389.75)
    m = 30000
    _say(f"free runs, {m} cycles: generic vs K = 4 sufficient-statistic theta steps")
    a = hbm.Sampler(wl, max_cycles=m)
    b = hbm.Sampler(wl, max_cycles=m, theta_substeps=4)
    a.run_cycles(m)
    b.run_cycles(m)
    ta, tb = a.theta_trace()[m // 5:], b.theta_trace()[m // 5:]
    for j in range(wl.p):
        ma, sa = batch_means(ta[:, j], MOMENT_BATCHES)
        mb, sb = batch_means(tb[:, j], MOMENT_BATCHES)
        z = abs(ma - mb) / math.hypot(sa, sb)
        _say(f"  theta[{j}] generic {ma:.5f}±{sa:.5f} K=4 {mb:.5f}±{sb:.5f} z={z:.2f}")
        assert z < 4.0
    a.close()
    b.close()


def test_argument_errors(hbm):
    wl = synth.bb1_lf(n=500, seed=88, chunk=500_000)
    with pytest.raises(hbm.HbmError, match="sufficient statistics"):
        hbm.Sampler(wl, max_cycles=10, theta_substeps=2)
    lf = synth.gamma_lf_1d(n=500, seed=89, fth=389.75)
    with pytest.raises(hbm.HbmError, match="theta_substeps"):
        hbm.Sampler(lf, max_cycles=10, theta_substeps=65)
    # a pool is one mode: datasets must match it
    pool = hbm.Pool(synth.GammaLF1D, capacity=4096, n_slots=2, max_cycles=10, stats_theta=True)
    with pytest.raises(hbm.HbmError, match="theta_substeps"):
        pool.admit([lf], [5])
    (slot,) = pool.admit([lf], [5], theta_substeps=3)
    assert slot is not None
    pool.close()
    plain = hbm.Pool(synth.GammaLF1D, capacity=4096, n_slots=2, max_cycles=10)
    with pytest.raises(hbm.HbmError, match="theta_substeps"):
        plain.admit([lf], [5], theta_substeps=2)
    plain.close()
    with pytest.raises(hbm.HbmError, match="sufficient statistics"):
        hbm.Pool(synth.bb1_lf(n=10, seed=1, chunk=100_000).model, capacity=1024, n_slots=1, max_cycles=10,
                 stats_theta=True)
