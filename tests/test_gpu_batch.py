"""GPU: batched and pooled datasets through the C ABI.

A dataset's chain depends only on its data, configuration and seed, so a
dataset advanced inside a batch (init_batch) or a continuously refilled pool
(create_pool / load_datasets / unload_dataset) must reproduce, bit for bit,
the chain of the same dataset run alone (whose parity with the FP64 oracle
is checked in test_gpu_parity.py).  The population log-likelihood of every
slot is also checked against the oracle directly.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FTH = 389.75   # threshold of the reference luminosity function (skips per-dataset calibration)


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


def _alone(hbm, wl, cycles, plain=False):
    s = hbm.Sampler(wl, max_cycles=max(cycles, 1))
    if plain:
        for _ in range(cycles):
            s.ram_sweep(1)
            s.theta_step()
    else:
        s.run_cycles(cycles)
    tr, chi = s.theta_trace(), s.state()[0]
    s.close()
    return tr, chi


def _lf_set(n_sets, seed0, n_lo, n_hi):
    rng = np.random.default_rng(seed0)
    ns = np.round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_sets))).astype(int)
    return [synth.gamma_lf_1d(n=int(n), seed=seed0 + j, fth=FTH) for j, n in enumerate(ns)]


def test_batch_matches_each_dataset_alone(hbm):
    wls = _lf_set(6, 700, 90, 3000) + [synth.gamma_lf_1d(n=256, seed=799, fth=FTH)]
    _say(f"batch of {len(wls)} LF datasets, N={[w.n for w in wls]}, 80 cycles (graph)")
    b = hbm.Batch(wls, max_cycles=80)
    b.run_cycles(80)
    for j, w in enumerate(wls):
        tr, chi = _alone(hbm, w, 80)
        assert np.array_equal(b.theta_trace(j), tr), j
        assert np.array_equal(b.latents(j), chi), j
    b.close()


def test_batch_plain_calls_nn3d(hbm):
    wls = [synth.normal_normal_3d(n=n, seed=s) for n, s in ((300, 5), (1000, 6), (77, 7))]
    _say("batch of 3 NN3D datasets, 30 plain sweep + theta-step cycles")
    b = hbm.Batch(wls, max_cycles=30)
    for _ in range(30):
        rates = b.ram_sweep(1, rate=True)
        assert rates.shape == (3,) and np.all((rates >= 0) & (rates <= 1))
        acc = b.theta_step()
        assert set(acc.tolist()) <= {0, 1}
    for j, w in enumerate(wls):
        tr, chi = _alone(hbm, w, 30, plain=True)
        assert np.array_equal(b.theta_trace(j), tr), j
        assert np.array_equal(b.latents(j), chi), j
    b.close()


def test_batch_pop_loglik_matches_oracle(hbm):
    wls = _lf_set(4, 900, 300, 5000)
    _say(f"batch pop_loglik, N={[w.n for w in wls]}")
    b = hbm.Batch(wls, max_cycles=20)
    b.run_cycles(20)
    thetas = np.array([w.theta_true for w in wls]) + np.array([0.01, -0.02])
    got = b.pop_loglik(thetas)
    for j, w in enumerate(wls):
        o = oracle.Oracle(w)
        chi = b.latents(j)
        ref = o.pop_loglik(thetas[j], chi)
        scale = np.sum(np.abs(o.pop_terms(thetas[j], chi)))
        assert abs(got[j] - ref) <= 1e-6 * scale + 1e-12 * w.n, (j, got[j], ref)
    b.close()


def test_pool_jobs_match_alone_runs(hbm):
    """Continuous batching: jobs admitted as space frees, stopped by their
    budgets on the device and retired; each job's samples equal its run alone."""
    wls = _lf_set(7, 1100, 200, 2500)
    budgets = [40, 70, 33, 90, 50, 21, 64]
    _say(f"pool: 7 jobs N={[w.n for w in wls]} budgets={budgets}, 3 slots, capacity 4608")
    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=4608, n_slots=3, max_cycles=100)
    pending = list(range(len(wls)))
    done = {}
    where = {}
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
        assert pool.resident, "a job larger than the empty pool"
        pool.run_cycles(16)
        rounds += 1
        for slot in pool.finished():
            j = where.pop(slot)
            info = pool.info(slot)
            assert info["n_theta"] == budgets[j] and info["k"] == budgets[j] and not info["active"]
            chi = pool.latents(slot)
            done[j] = (pool.retire(slot), chi)
        assert rounds < 100
    assert sorted(done) == list(range(len(wls)))
    for j, w in enumerate(wls):
        tr, chi = _alone(hbm, w, budgets[j])
        assert np.array_equal(done[j][0], tr), j
        assert np.array_equal(done[j][1], chi), j
    pool.close()


def test_pool_launch_extent_follows_the_last_job(hbm):
    """Cycles launch only up to the last loaded slot and occupied tile: the
    extent shrinks when the highest job retires and grows when a later job
    lands beyond it; every job still equals its run alone."""
    wls = [synth.gamma_lf_1d(n=n, seed=1500 + j, fth=FTH) for j, n in enumerate((3000, 1200, 2600, 5000))]
    budgets = [72, 48, 16, 32]
    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=65536, n_slots=6, max_cycles=100)
    sa, sb, sc = pool.admit(wls[:3], budgets[:3])
    pool.run_cycles(16)                       # the third job (highest slot and tiles) finishes here
    assert pool.finished() == [sc]
    done = {2: (pool.retire(sc), None)}
    pool.run_cycles(8)                        # extent: the first two jobs only
    (sd,) = pool.admit([wls[3]], [budgets[3]])
    pool.run_cycles(40)                       # extent grows again to the new job
    for slot, j in ((sb, 1), (sd, 3)):
        assert slot in pool.finished()
        done[j] = (pool.retire(slot), None)
    pool.run_cycles(16)
    assert pool.finished() == [sa]
    done[0] = (pool.retire(sa), None)
    for j, w in enumerate(wls):
        tr, _ = _alone(hbm, w, budgets[j])
        assert np.array_equal(done[j][0], tr), j
    pool.close()


def test_pool_rejects_bad_loads(hbm):
    _say("pool: invalid placements and slots are rejected, the pool stays usable")
    w = synth.gamma_lf_1d(n=300, seed=3, fth=FTH)
    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=1024, n_slots=2, max_cycles=10)
    cfg = hbm.make_config(w, max_cycles=10)
    th0 = np.array([w.theta0])
    with pytest.raises(hbm.HbmError, match="multiple of 256"):
        hbm.load_datasets(pool.ctx, [0], [100], [cfg], th0)
    with pytest.raises(hbm.HbmError, match="slot out of range"):
        hbm.load_datasets(pool.ctx, [5], [0], [cfg], th0)
    with pytest.raises(hbm.HbmError, match="budget"):
        hbm.load_datasets(pool.ctx, [0], [0], [cfg], th0, [11])
    with pytest.raises(hbm.HbmError, match="capacity"):
        hbm.load_datasets(pool.ctx, [0], [768], [cfg], th0)
    (slot,) = pool.admit([w], [10])
    other = 1 - slot
    with pytest.raises(hbm.HbmError, match="overlaps"):
        hbm.load_datasets(pool.ctx, [other], [pool.resident[slot][0]], [cfg], th0)
    with pytest.raises(hbm.HbmError, match="already holds"):
        hbm.load_datasets(pool.ctx, [slot], [512], [cfg], th0)
    pool.run_cycles(10)
    assert pool.finished() == [slot]
    tr = pool.retire(slot)
    ref, _ = _alone(hbm, w, 10)
    assert np.array_equal(tr, ref)
    with pytest.raises(hbm.HbmError, match="no dataset"):
        hbm.get_stats(pool.ctx, slot)
    pool.close()


@pytest.mark.parametrize("make", [lambda: synth.gamma_lf_1d(n=5000, seed=71, fth=FTH),
                                  lambda: synth.normal_normal_3d(n=1500, seed=8)], ids=["lf1d", "nn3d"])
def test_launch_shape_does_not_change_the_chain(hbm, make):
    wl = make()
    _say(f"launch shapes 1/2/4 tiles per workgroup, {wl.name} N={wl.n}")
    ref, ref_chi = _alone(hbm, wl, 70)
    for tpw in (2, 4):
        s = hbm.Sampler(wl, max_cycles=70)
        s.set_launch(tpw)
        s.run_cycles(70)
        assert np.array_equal(s.theta_trace(), ref), tpw
        assert np.array_equal(s.state()[0], ref_chi), tpw
        s.close()


def test_full_batch_sampled_datasets(hbm):
    """The 256-catalog batch at its full size (sum N ~ 6e6), autotuned and
    graph-replayed as the bench runs it: the smallest, the largest and a
    middle dataset equal, bit for bit, the same datasets run alone, and the
    largest one's population log-likelihood matches the oracle at the batch's
    latents."""
    wls = synth.gamma_lf_batch(256)
    ns = np.array([w.n for w in wls])
    _say(f"full batch: 256 datasets, sum N = {ns.sum()}")
    trial, cycles = 8, 30
    total = hbm.autotune_cycles(trial) + cycles
    b = hbm.Batch(wls, max_cycles=total)
    pick, _ = b.autotune(trial)
    b.run_cycles(cycles)
    picks = sorted({int(np.argmin(ns)), int(np.argmax(ns)), int(np.argsort(ns)[len(ns) // 2])})
    for j in picks:
        _say(f"  dataset {j}: N = {wls[j].n}, shape {pick}")
        tr, chi = _alone(hbm, wls[j], total)
        assert np.array_equal(b.theta_trace(j), tr), j
        assert np.array_equal(b.latents(j), chi), j
    j = int(np.argmax(ns))
    th = np.array([w.theta_true for w in wls])
    got = b.pop_loglik(th)
    o = oracle.Oracle(wls[j])
    chi = b.latents(j)
    ref = o.pop_loglik(th[j], chi)
    scale = np.sum(np.abs(o.pop_terms(th[j], chi)))
    assert abs(got[j] - ref) <= 1e-6 * scale + 1e-12 * wls[j].n, (got[j], ref)
    b.close()


def test_autotune_batch_keeps_chains(hbm):
    wls = _lf_set(5, 1300, 300, 4000)
    _say(f"autotune on a batch N={[w.n for w in wls]}")
    total = hbm.autotune_cycles(8) + 10
    b = hbm.Batch(wls, max_cycles=total)
    pick, us = b.autotune(8)
    _say(f"  choice {pick}; us/cycle {dict(zip(hbm.tune_labels(), np.round(us, 2)))}")
    assert pick["tiles_per_group"] in (1, 2, 4) and pick["groups_per_cu"] in (0, 4, 2)
    assert not pick["persistent"]                  # a batch takes graphs: the persistent launch is not timed
    assert np.all(us[:9] > 0) and np.isnan(us[9])
    b.run_cycles(10)
    for j, w in enumerate(wls):
        tr, chi = _alone(hbm, w, total)
        assert np.array_equal(b.theta_trace(j), tr), j
        assert np.array_equal(b.latents(j), chi), j
    b.close()


def test_request_loop_results_same_alone_and_in_the_mix(hbm):
    """The serving loop over the GPU pool: jobs arriving over time, admitted
    by memory, batched continuously; each job's theta trace equals its run alone."""
    from paper_2105_08026_amd import serve as sv
    # the first two jobs arrive together and fit side by side (15 of the
    # pool's 16 tiles), so they are resident at the same time; the third
    # waits for tiles, the later ones arrive while others run
    specs = [(0.00, 3100, 900, 192), (0.00, 3101, 2600, 160), (0.00, 3102, 300, 64),
             (0.002, 3103, 1700, 128), (0.004, 3104, 2500, 64), (0.02, 3105, 700, 32)]
    jobs = [sv.Job(i, t, seed, n, sw) for i, (t, seed, n, sw) in enumerate(specs)]
    _say(f"request loop: {len(jobs)} jobs into a 4096-object, 3-slot pool")

    def make(job):
        return synth.gamma_lf_1d(n=job.n, seed=job.seed, fth=FTH)

    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=4096, n_slots=3, max_cycles=200)
    res = sv.serve(jobs, sv.PoolExecutor(pool, make, chunk=16))
    pool.close()
    assert len(res["jobs"]) == len(jobs) and res["p99_s"] >= res["p50_s"] > 0
    # jobs really shared the device: some were resident together
    fin = res["jobs"]
    overlapping = sum(1 for a in fin for b in fin if a.id < b.id and a.admitted < b.done and b.admitted < a.done)
    _say(f"  mean resident {res['mean_resident']:.2f}, overlapping job pairs {overlapping}")
    assert res["mean_resident"] > 1.0 and overlapping >= 1
    for j in res["jobs"]:
        tr, _ = _alone(hbm, make(j), j.sweeps)
        assert np.array_equal(j.trace, tr), j.id


def test_request_loop_streams_each_jobs_snapshots(hbm):
    """Serving with streamed latent snapshots: a pool with a ring of two
    chunks of rows; every job's snapshots reach the host as they are taken
    and equal the snapshots of the job run alone."""
    from paper_2105_08026_amd import serve as sv
    specs = [(0.00, 3200, 900, 96), (0.01, 3201, 2600, 64), (0.03, 3202, 300, 80), (0.06, 3203, 1500, 48)]
    jobs = [sv.Job(i, t, seed, n, sw) for i, (t, seed, n, sw) in enumerate(specs)]
    thin, chunk = 4, 16
    rows = {}

    def make(job):
        return synth.gamma_lf_1d(n=job.n, seed=job.seed, fth=FTH)

    def on_rows(job, first, r):
        rows.setdefault(job.id, []).append((first, r))
    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=4096, n_slots=3, max_cycles=200, snap_rows=2 * (chunk // thin))
    res = sv.serve(jobs, sv.PoolExecutor(pool, make, chunk=chunk, cfg={"thin": thin}, on_rows=on_rows))
    pool.close()
    assert len(res["jobs"]) == len(jobs)
    for j in res["jobs"]:
        alone = hbm.Sampler(make(j), max_cycles=j.sweeps, thin=thin)
        alone.run_cycles(j.sweeps)
        ref = alone.chi_snapshots(0, j.sweeps // thin)
        got = np.concatenate([r for _, r in rows[j.id]])
        assert [f for f, _ in rows[j.id]][0] == 0 and np.array_equal(got, ref), j.id
        assert np.array_equal(j.trace, alone.theta_trace()), j.id
        alone.close()


@pytest.mark.parametrize("make", [lambda: synth.gamma_lf_1d(n=3000, seed=72, fth=FTH),
                                  lambda: synth.normal_normal_3d(n=700, seed=9)], ids=["lf1d", "nn3d"])
def test_checkpoint_resume_continues_exactly(hbm, make):
    wl = make()
    _say(f"checkpoint after 40 cycles, resume in a new context, 37 more: {wl.name} N={wl.n}")
    a = hbm.Sampler(wl, max_cycles=100)
    a.run_cycles(40)
    ck = a.checkpoint()
    a.run_cycles(37)
    ref_tr, ref_chi = a.theta_trace(), a.state()[0]
    a.close()
    b = hbm.Sampler(wl, max_cycles=100)
    b.restore(ck)
    assert b.theta()[2] == 40 and hbm.n_theta_samples(b.ctx) == 40
    b.run_cycles(37)
    assert np.array_equal(b.theta_trace(), ref_tr)
    assert np.array_equal(b.state()[0], ref_chi)
    other = hbm.Sampler(synth.gamma_lf_1d(n=2000, seed=73, fth=FTH), max_cycles=100)
    with pytest.raises(hbm.HbmError, match="differently shaped|different dataset"):
        hbm.set_state(other.ctx, ck[0])
    other.close()
    b.close()


def test_batch_checkpoint_resume(hbm):
    wls = _lf_set(4, 1500, 300, 3000)
    _say(f"batch checkpoint/resume, N={[w.n for w in wls]}")
    a = hbm.Batch(wls, max_cycles=90)
    a.run_cycles(33)
    blob = hbm.get_state(a.ctx)
    torch.cuda.synchronize()
    bufs = [t.clone() for t in (a.chi, a.chol, a.acc)]
    a.run_cycles(50)
    ref = [a.theta_trace(j) for j in range(len(wls))]
    b = hbm.Batch(wls, max_cycles=90)
    with torch.no_grad():
        for dst, src in zip((b.chi, b.chol, b.acc), bufs):
            dst.copy_(src)
    torch.cuda.synchronize()
    hbm.set_state(b.ctx, blob)
    b.run_cycles(50)
    for j in range(len(wls)):
        assert np.array_equal(b.theta_trace(j), ref[j]), j
    a.close()
    b.close()
