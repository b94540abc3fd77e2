"""Fused cycles in contexts with several datasets (batches and pools): every
tile's workgroup takes its own dataset's theta step from that dataset's tile
partials, and each dataset's side workgroup writes its state.  Chains must be
bit for bit those of the two-kernel cycle -- every dataset's theta trace,
latents, factors and counters -- with datasets of one partial tile to many
tiles, with budgets that stop datasets inside a graph while others go on,
with jobs admitted between runs, and with theta sub-steps from sufficient
statistics.
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


def _lf_set(n_sets, seed0, n_lo, n_hi):
    rng = np.random.default_rng(seed0)
    ns = np.round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_sets))).astype(int)
    return [synth.gamma_lf_1d(n=int(n), seed=seed0 + j, fth=FTH) for j, n in enumerate(ns)]


def _same_batches(a, b):
    for j in range(a.n_datasets):
        assert np.array_equal(a.theta_trace(j), b.theta_trace(j)), j
        assert np.array_equal(a.latents(j), b.latents(j)), j
        sa, sb = a.stats(j), b.stats(j)
        for key in sa:
            assert sa[key] == sb[key] or (np.isnan(sa[key]) and np.isnan(sb[key])), (j, key)
        ta, ca, ka = a.theta(j)
        tb, cb, kb = b.theta(j)
        assert ka == kb and np.array_equal(ta, tb) and np.array_equal(ca, cb), j
    # every dataset's latents, factors and counters in the packed buffers
    # (the padding between datasets is never written)
    torch.cuda.synchronize()
    for o, n in zip(a.offsets, a.ns):
        for x, y in ((a.chi, b.chi), (a.chol, b.chol), (a.acc, b.acc)):
            assert torch.equal(x[..., o:o + n], y[..., o:o + n])


BATCHES = {
    "lf1d": lambda: _lf_set(6, 900, 90, 5000) + [synth.gamma_lf_1d(n=256, seed=999, fth=FTH)],
    "nn1d": lambda: [synth.normal_normal_1d(n=n, seed=40 + j) for j, n in enumerate((300, 1000, 17, 2600))],
    "lf3d": lambda: [synth.gamma_lf_3d(n=n, seed=50 + j, fth=FTH) for j, n in enumerate((700, 2100, 300))],
    "nn3d": lambda: [synth.normal_normal_3d(n=n, seed=60 + j) for j, n in enumerate((500, 257))],
    "bb1": lambda: [synth.bb1_lf(n=n, seed=70 + j, chunk=1_000_000) for j, n in enumerate((900, 3000))],
    "tiny": lambda: [synth.gamma_lf_1d(n=n, seed=90 + j, fth=FTH) for j, n in enumerate((1, 2, 257))],
}


@pytest.mark.parametrize("name", list(BATCHES))
def test_fused_batch_equals_two_kernel_cycles(hbm, name):
    wls = BATCHES[name]()
    cycles = 120
    _say(f"fused batch vs two-kernel cycles: {name}, N={[w.n for w in wls]}, {cycles} cycles in calls of 1, 40 and 79")
    a = hbm.Batch(wls, max_cycles=cycles)
    a.set_cycle_mode(hbm.HBM_CYCLES_FUSED)
    for n in (1, 40, 79):
        a.run_cycles(n)
    lc = a.launch_counts()
    assert lc["replayed_cycles"] == cycles, lc
    b = hbm.Batch(wls, max_cycles=cycles)
    b.run_cycles(cycles, use_graph=False)
    _same_batches(a, b)
    a.close()
    b.close()


def test_fused_batch_tile_shape_is_ignored(hbm):
    """A multi-dataset context runs one tile per workgroup in fused mode
    whatever the launch shape; the chain is unchanged."""
    wls = _lf_set(4, 950, 200, 3000)
    _say(f"fused batch with launch shape 4: N={[w.n for w in wls]}, 70 cycles")
    a = hbm.Batch(wls, max_cycles=70)
    a.set_cycle_mode(hbm.HBM_CYCLES_FUSED)
    a.set_launch(4)
    a.run_cycles(70)
    b = hbm.Batch(wls, max_cycles=70)
    b.run_cycles(70, use_graph=False)
    _same_batches(a, b)


@pytest.mark.parametrize("make", [lambda: _lf_set(3, 960, 300, 4000),
                                  lambda: [synth.normal_normal_3d(n=n, seed=80 + j) for j, n in enumerate((900, 300))]])
def test_fused_batch_theta_substeps(hbm, make):
    wls = make()
    _say(f"fused batch, 3 theta steps per cycle from sufficient statistics: {wls[0].name} N={[w.n for w in wls]}")
    a = hbm.Batch(wls, max_cycles=60, theta_substeps=3)
    a.set_cycle_mode(hbm.HBM_CYCLES_FUSED)
    a.run_cycles(60)
    b = hbm.Batch(wls, max_cycles=60, theta_substeps=3)
    b.run_cycles(60, use_graph=False)
    _same_batches(a, b)


def _alone(hbm, wl, cycles):
    s = hbm.Sampler(wl, max_cycles=max(cycles, 1))
    s.run_cycles(cycles, use_graph=False)
    tr, chi = s.theta_trace(), s.state()[0]
    s.close()
    return tr, chi


def test_fused_pool_budgets_and_admissions(hbm):
    """Continuous batching in fused mode: budgets stop datasets inside a graph
    while others go on, jobs are admitted between runs; every job's trace and
    latents equal its run alone."""
    wls = _lf_set(7, 1200, 200, 2500)
    budgets = [40, 70, 33, 90, 50, 21, 64]
    _say(f"fused pool: 7 jobs N={[w.n for w in wls]} budgets={budgets}, 3 slots, capacity 4608")
    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=4608, n_slots=3, max_cycles=100)
    hbm.set_cycle_mode(pool.ctx, hbm.HBM_CYCLES_FUSED)
    pending = list(range(len(wls)))
    done, where = {}, {}
    rounds = 0
    while pending or pool.resident:
        while pending:
            j = pending[0]
            if not pool.fits(wls[j].n):
                break
            slot = pool.admit([wls[j]], [budgets[j]])[0]
            assert slot is not None
            where[slot] = j
            pending.pop(0)
        assert pool.resident
        pool.run_cycles(16)
        rounds += 1
        for slot in pool.finished():
            j = where.pop(slot)
            info = pool.info(slot)
            assert info["n_theta"] == budgets[j] and not info["active"]
            chi = pool.latents(slot)
            done[j] = (pool.retire(slot), chi)
        assert rounds < 100
    assert sorted(done) == list(range(len(wls)))
    for j, w in enumerate(wls):
        tr, chi = _alone(hbm, w, budgets[j])
        assert np.array_equal(done[j][0], tr), j
        assert np.array_equal(done[j][1], chi), j
    pool.close()


def test_autotune_times_fused_on_a_batch(hbm):
    wls = _lf_set(5, 1300, 300, 3000)
    b = hbm.Batch(wls, max_cycles=hbm.autotune_cycles(8) + 30)
    pick, us = b.autotune(8)
    labels = hbm.tune_labels()
    _say(f"batch autotune choice {pick}; us/cycle {dict(zip(labels, np.round(us, 2)))}")
    timed = {lab: u for lab, u in zip(labels, us)}
    assert np.isfinite(timed["fused_tpw1"]) and timed["fused_tpw1"] > 0
    assert np.isnan(timed["fused_tpw2"]) and np.isnan(timed["fused_tpw4"])
    b.run_cycles(30)
    c = hbm.Batch(wls, max_cycles=hbm.autotune_cycles(8) + 30)
    c.run_cycles(hbm.autotune_cycles(8) + 30, use_graph=False)
    _same_batches(b, c)
