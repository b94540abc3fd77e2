"""Fused cycles (mode HBM_CYCLES_FUSED: after the first sweep, one launch per
cycle in which every workgroup takes the previous sweep's theta step itself
and then sweeps its tiles) against the two-kernel cycle as plain launches:
chains must be bit for bit the same -- latents, factors, counters, the theta
trace and the library's chain state -- for every model, at sizes from one
partial tile to the 300,000-object catalog, with one, two and four tiles per
workgroup, with snapshots, with theta sub-steps from sufficient statistics,
and with a budget that stops the dataset inside a graph.
"""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FTH = 389.75


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


def _same(a, b):
    assert np.array_equal(a.theta_trace(), b.theta_trace())
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    sa, sb = a.stats(), b.stats()
    for key in sa:
        assert sa[key] == sb[key] or (np.isnan(sa[key]) and np.isnan(sb[key])), key
    ta, ca, ka = a.theta()
    tb, cb, kb = b.theta()
    assert ka == kb and np.array_equal(ta, tb) and np.array_equal(ca, cb)


MODELS = {
    "nn1d_1000": lambda: synth.normal_normal_1d(n=1000, seed=0),
    "lf1d_3001": lambda: synth.gamma_lf_1d(n=3001, seed=91, fth=FTH),
    "lf1d_100": lambda: synth.gamma_lf_1d(n=100, seed=92, fth=FTH),
    "lf1d_70000": lambda: synth.gamma_lf_1d(n=70000, seed=93, fth=FTH),
    "lf3d_5000": lambda: synth.gamma_lf_3d(n=5000, seed=94, fth=FTH),
    "nn3d_777": lambda: synth.normal_normal_3d(n=777, seed=5),
    "bb1_4000": lambda: synth.bb1_lf(n=4000, seed=95, chunk=1_000_000),
}


def _fused(hbm, wl, max_cycles, tpw=1, **kw):
    s = hbm.Sampler(wl, max_cycles=max_cycles, **kw)
    s.set_cycle_mode(hbm.HBM_CYCLES_FUSED)
    s.set_launch(tpw)
    return s


@pytest.mark.parametrize("name", list(MODELS))
def test_fused_equals_two_kernel_cycles(hbm, name):
    wl = MODELS[name]()
    cycles = 150
    _say(f"fused vs two-kernel cycles: {name} N={wl.n}, {cycles} cycles in calls of 1, 37 and 112")
    a = _fused(hbm, wl, cycles)
    for n in (1, 37, 112):
        a.run_cycles(n)
    lc = a.launch_counts()
    assert lc["persistent_cycles"] == 0 and lc["replayed_cycles"] == cycles, lc
    b = hbm.Sampler(wl, max_cycles=cycles)
    b.run_cycles(cycles, use_graph=False)
    _same(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("tpw", [2, 4])
def test_fused_tiles_per_workgroup(hbm, tpw):
    wl = synth.gamma_lf_1d(n=9000, seed=100, fth=FTH)      # 36 tiles: ragged for 4 per workgroup
    _say(f"fused cycles with {tpw} tiles per workgroup: N={wl.n}, 70 cycles")
    a = _fused(hbm, wl, 70, tpw=tpw)
    a.run_cycles(70)
    b = hbm.Sampler(wl, max_cycles=70)
    b.run_cycles(70, use_graph=False)
    _same(a, b)


def test_fused_full_catalog(hbm):
    wl = synth.gamma_lf_1d()
    _say(f"fused vs two-kernel graph replay: N={wl.n}, 70 cycles")
    a = _fused(hbm, wl, 70)
    a.run_cycles(70)
    b = hbm.Sampler(wl, max_cycles=70)
    b.set_cycle_mode(hbm.HBM_CYCLES_GRAPH)
    b.run_cycles(70)
    _same(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("tpw", [1, 2])
def test_fused_snapshots(hbm, tpw):
    wl = synth.gamma_lf_1d(n=2600, seed=96, fth=FTH)
    _say(f"fused cycles with latent snapshots every 7 sweeps, {tpw} tiles per workgroup")
    a = _fused(hbm, wl, 100, tpw=tpw, thin=7)
    a.run_cycles(60)
    a.run_cycles(40)
    b = hbm.Sampler(wl, max_cycles=100, thin=7)
    b.run_cycles(100, use_graph=False)
    _same(a, b)
    assert np.array_equal(a.chi_snapshots(0, 14), b.chi_snapshots(0, 14))


@pytest.mark.parametrize("tpw", [1, 2])
@pytest.mark.parametrize("make", [lambda: synth.gamma_lf_1d(n=4000, seed=97, fth=FTH),
                                  lambda: synth.normal_normal_3d(n=900, seed=6)])
def test_fused_theta_substeps(hbm, make, tpw):
    wl = make()
    _say(f"fused cycles, 4 theta steps per cycle from sufficient statistics: {wl.name} N={wl.n}, {tpw} tiles per workgroup")
    a = _fused(hbm, wl, 80, tpw=tpw, theta_substeps=4)
    a.run_cycles(80)
    b = hbm.Sampler(wl, max_cycles=80, theta_substeps=4)
    b.run_cycles(80, use_graph=False)
    _same(a, b)


def test_fused_stops_at_the_budget(hbm):
    """A one-slot pool whose dataset fills it is a one-dataset context: its
    budget stops the chain inside a graph of fused cycles."""
    wl = synth.gamma_lf_1d(n=1280, seed=98, fth=FTH)
    _say("fused cycles with a budget of 45 inside 80 graph cycles")
    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=wl.n, n_slots=1, max_cycles=80)
    (slot,) = pool.admit([wl], [45])
    hbm.set_cycle_mode(pool.ctx, hbm.HBM_CYCLES_FUSED)
    pool.run_cycles(80)
    assert pool.info(slot)["n_theta"] == 45 and pool.info(slot)["active"] == 0
    got = pool.theta_trace(slot)
    lat = pool.latents(slot)
    s = hbm.Sampler(wl, max_cycles=45)
    s.run_cycles(45, use_graph=False)
    assert np.array_equal(got, s.theta_trace())
    assert np.array_equal(lat, s.state()[0])
    pool.close()


def test_autotune_times_fused_candidates(hbm):
    wl = synth.gamma_lf_1d(n=20000, seed=101, fth=FTH)
    s = hbm.Sampler(wl, max_cycles=hbm.autotune_cycles(8) + 40)
    pick, us = s.autotune(8)
    labels = hbm.tune_labels()
    _say(f"autotune choice {pick}; us/cycle {dict(zip(labels, np.round(us, 2)))}")
    for lab, u in zip(labels, us):
        if lab.startswith("fused") or lab.startswith("tpw"):
            assert np.isfinite(u) and u > 0, lab
    # whatever it picked, the chain goes on as the plain cycle would
    s.run_cycles(40)
    b = hbm.Sampler(wl, max_cycles=hbm.autotune_cycles(8) + 40)
    b.run_cycles(hbm.autotune_cycles(8) + 40, use_graph=False)
    _same(s, b)
