"""GPU tests of the streamed sampler (latent snapshots to the host as they are
taken, through a small device ring).

* every snapshot of a streamed run equals, bit for bit, the snapshot a plain
  run keeps in a full device buffer, for FP32 1-D and FP64 3-D latents, with
  chunk lengths and thinning that make the ring wrap inside a chunk;
* the theta chain is unchanged by streaming;
* a pool streams each resident job's snapshots (jobs admitted at different
  sweeps, one stopped by its budget mid-chunk) equal to each job run alone;
* the library's file-descriptor sink writes the same rows to a file;
* a ring in pinned host memory (the sweep writes the snapshots through its
  device mapping) streams the same rows, with no copies;
* the sink can stop a run; a ring smaller than two chunks is refused.
"""
import sys

import numpy as np
import pytest

import synth

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


@pytest.mark.parametrize("make,thin,chunk,m", [
    (lambda: synth.gamma_lf_1d(n=5000, seed=91, fth=389.75), 3, 16, 200),
    (lambda: synth.gamma_lf_1d(n=777, seed=92, fth=389.75), 7, 20, 300),
    (lambda: synth.normal_normal_3d(n=1500, seed=93), 2, 33, 150),
])
def test_streamed_snapshots_equal_the_full_buffer(hbm, make, thin, chunk, m):
    wl = make()
    ring = 2 * (-(-chunk // thin))
    _say(f"streaming N={wl.n} d={wl.d} thin={thin} chunk={chunk} ring={ring} rows, {m} cycles")
    full = hbm.Sampler(wl, max_cycles=m, thin=thin)
    full.run_cycles(m)
    ref = full.chi_snapshots(0, m // thin)
    st = hbm.Sampler(wl, max_cycles=m, thin=thin, snap_rows=ring)
    got = st.run_streamed(m, chunk)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
    assert np.array_equal(st.theta_trace(), full.theta_trace())
    assert st.snaps.shape[0] == ring
    full.close()
    st.close()


def test_pool_streams_each_job(hbm):
    jobs = [synth.gamma_lf_1d(n=n, seed=94 + j, fth=389.75) for j, n in enumerate((900, 2300, 400))]
    thin, chunk = 4, 12
    ring = 2 * (-(-chunk // thin))
    budgets = [70, 0, 45]
    pool = hbm.Pool(synth.GammaLF1D, capacity=4096, n_slots=3, max_cycles=200, snap_rows=ring)
    rows = {}

    def sink(slot, first, r):
        rows.setdefault(slot, []).append((first, r))
        return False
    (s0,) = pool.admit([jobs[0]], [budgets[0]], thin=thin)
    pool.run_streamed(20, chunk, sink)
    s1, s2 = pool.admit(jobs[1:], budgets[1:], thin=thin)
    pool.run_streamed(100, chunk, sink)
    for slot, w, b, cycles in ((s0, jobs[0], budgets[0], 120), (s1, jobs[1], budgets[1], 100),
                               (s2, jobs[2], budgets[2], 100)):
        done = min(cycles, b) if b > 0 else cycles
        alone = hbm.Sampler(w, max_cycles=done, thin=thin)
        alone.run_cycles(done)
        ref = alone.chi_snapshots(0, done // thin)
        firsts = [f for f, _ in rows[slot]]
        got = np.concatenate([r for _, r in rows[slot]])
        assert firsts[0] == 0 and got.shape == ref.shape, (slot, firsts, got.shape, ref.shape)
        assert np.array_equal(got, ref), slot
        alone.close()
    pool.close()


def test_sink_stops_and_ring_checks(hbm):
    wl = synth.gamma_lf_1d(n=1000, seed=97, fth=389.75)
    s = hbm.Sampler(wl, max_cycles=400, thin=2, snap_rows=8)
    seen = []
    with pytest.raises(hbm.HbmError, match="stopped"):
        s.run_streamed(400, 8, lambda first, rows: seen.append(first) or first >= 8)
    assert seen and seen[-1] >= 8
    with pytest.raises(hbm.HbmError, match="snap_rows"):
        s.run_streamed(40, 9)           # ceil(9 / 2) = 5 rows per chunk: a ring of 8 is too small
    s.close()


def test_file_sink(hbm, tmp_path):
    wl = synth.gamma_lf_1d(n=3000, seed=98, fth=389.75)
    m, thin, chunk = 120, 5, 30
    full = hbm.Sampler(wl, max_cycles=m, thin=thin)
    full.run_cycles(m)
    ref = full.chi_snapshots(0, m // thin)
    s = hbm.Sampler(wl, max_cycles=m, thin=thin, snap_rows=12)
    path = str(tmp_path / "chi.f32")
    s.run_to_file(m, chunk, path)
    got = np.fromfile(path, dtype=np.float32).reshape(-1, wl.d, wl.n)
    assert np.array_equal(got, ref)
    full.close()
    s.close()


@pytest.mark.parametrize("make,thin,chunk,m", [
    (lambda: synth.gamma_lf_1d(n=5000, seed=99, fth=389.75), 3, 16, 200),
    (lambda: synth.normal_normal_3d(n=700, seed=100), 5, 21, 160),
])
def test_host_ring(hbm, make, thin, chunk, m):
    wl = make()
    ring = 2 * (-(-chunk // thin))
    full = hbm.Sampler(wl, max_cycles=m, thin=thin)
    full.run_cycles(m)
    ref = full.chi_snapshots(0, m // thin)
    hs = hbm.Sampler(wl, max_cycles=m, thin=thin, snap_rows=ring, snap_host=True)
    assert not hs.snaps.is_cuda and hs.snaps.is_pinned()
    got = hs.run_streamed(m, chunk)
    assert np.array_equal(got, ref)
    assert np.array_equal(hs.theta_trace(), full.theta_trace())
    full.close()
    hs.close()
    # a plain run with the host buffer keeps the first rows, read back by get_samples
    hp = hbm.Sampler(wl, max_cycles=m, thin=thin, snap_host=True)
    hp.run_cycles(m)
    assert np.array_equal(hp.chi_snapshots(0, m // thin), ref)
    hp.close()
