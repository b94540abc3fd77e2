"""The request loop's host logic on a simulated executor (no GPU).

The simulated pool has the real admission rule (a free slot and a
contiguous run of free 256-object tiles, first fit), advances every
resident job by one chunk of cycles per step on a virtual clock, and
finishes a job exactly at its sweep budget, as the device does.
"""
import numpy as np
import pytest

from paper_2105_08026_amd.serve import Job, TileAllocator, serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class SimExecutor:
    def __init__(self, clock, n_tiles, n_slots, chunk=32, max_cycles=5000, t_fixed=9e-6, t_obj=2.5e-11):
        self.clock, self.chunk, self.max_cycles = clock, chunk, max_cycles
        self.alloc = TileAllocator(n_tiles)
        self.free = list(range(n_slots))
        self.left = {}
        self.n = {}
        self.t_fixed, self.t_obj = t_fixed, t_obj
        self.admit_log = []
        self.max_resident_tiles = 0

    def fits(self, job):
        return bool(self.free) and self.alloc.find(-(-job.n // 256)) is not None

    def too_big(self, job):
        return -(-job.n // 256) > self.alloc.owner.size or job.sweeps > self.max_cycles

    def admit(self, job, wl):
        nt = -(-job.n // 256)
        start = self.alloc.find(nt)
        slot = self.free.pop(0)
        self.alloc.take(start, nt, slot)
        self.left[slot], self.n[slot] = job.sweeps, job.n
        self.admit_log.append(job.id)
        self.max_resident_tiles = max(self.max_resident_tiles, self.alloc.owner.size - self.alloc.free_tiles)
        return slot

    def run(self):
        objs = sum(self.n[s] for s in self.left if self.left[s] > 0)
        self.clock.t += self.chunk * (self.t_fixed + self.t_obj * objs)
        out = []
        for s in list(self.left):
            if self.left[s] > 0:
                self.left[s] -= self.chunk
                if self.left[s] <= 0:
                    out.append(s)
        return out

    def retire(self, slot):
        self.alloc.release(slot)
        self.free.append(slot)
        sweeps = self.left.pop(slot)
        self.n.pop(slot)
        return np.zeros((0, 2)) if sweeps <= 0 else None


def poisson_jobs(rate, horizon, seed, n_lo=1e3, n_hi=3e5, sweeps=(1000, 2000, 5000)):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > horizon:
            return out
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        out.append(Job(len(out), t, 10000 + len(out), n, int(rng.choice(sweeps))))


def test_allocator_first_fit_and_release():
    a = TileAllocator(10)
    assert a.find(4) == 0
    a.take(0, 4, 7)
    a.take(4, 3, 8)
    assert a.find(4) is None and a.find(3) == 7
    a.release(7)
    assert a.find(4) == 0 and a.free_tiles == 7
    with pytest.raises(AssertionError):
        a.take(3, 2, 9)


def test_every_job_finishes_fifo_with_budgets():
    clk = Clock()
    jobs = poisson_jobs(20.0, 30.0, seed=4)
    ex = SimExecutor(clk, n_tiles=4096, n_slots=16)
    res = serve(jobs, ex, make=lambda j: None, clock=clk, sleep=clk.sleep, prefetch=False)
    assert len(res["jobs"]) == len(jobs)
    # first come, first served
    assert ex.admit_log == sorted(ex.admit_log)
    for j in res["jobs"]:
        assert j.admitted >= j.arrival and j.done > j.admitted
        # a job cannot finish faster than its sweeps at the fixed per-cycle cost
        assert j.done - j.admitted >= j.sweeps * ex.t_fixed * 0.999
    assert res["p99_s"] >= res["p50_s"] > 0
    assert res["jobs_per_hour"] > 0


def test_memory_admission_queues_when_full():
    clk = Clock()
    # three jobs of 1000 tiles each into a 2048-tile pool: the third waits
    jobs = [Job(i, 0.0, i, 256000, 64) for i in range(3)]
    ex = SimExecutor(clk, n_tiles=2048, n_slots=8)
    res = serve(jobs, ex, make=lambda j: None, clock=clk, sleep=clk.sleep, prefetch=False)
    by = {j.id: j for j in res["jobs"]}
    assert by[0].admitted == by[1].admitted == 0.0
    assert by[2].admitted >= by[0].done
    assert ex.max_resident_tiles <= 2048


def test_job_larger_than_pool_is_rejected():
    clk = Clock()
    ex = SimExecutor(clk, n_tiles=16, n_slots=2)
    with pytest.raises(ValueError, match="never fit"):
        serve([Job(0, 0.0, 0, 5000, 32)], ex, make=lambda j: None, clock=clk, sleep=clk.sleep, prefetch=False)


def test_slots_limit_concurrency():
    clk = Clock()
    jobs = [Job(i, 0.0, i, 1000, 32 * (i + 1)) for i in range(6)]
    ex = SimExecutor(clk, n_tiles=4096, n_slots=2)
    res = serve(jobs, ex, make=lambda j: None, clock=clk, sleep=clk.sleep, prefetch=False)
    t = sorted([(j.admitted, 1) for j in res["jobs"]] + [(j.done, -1) for j in res["jobs"]],
               key=lambda x: (x[0], x[1]))
    live = np.cumsum([d for _, d in t])
    assert live.max() <= 2


class _ModePool:
    """Stands in for a Pool in PoolExecutor: records cycle-mode changes."""

    def __init__(self):
        self.tiles = np.full(64, -1)
        self.max_cycles = 1000
        self.device = "cpu"
        self.modes = []
        self.next_slot = 0

    def set_cycle_mode(self, mode):
        self.modes.append(mode)

    def fits(self, n):
        return True

    def admit(self, wls, budgets, **kw):
        self.next_slot += 1
        return [self.next_slot - 1]

    def run_cycles(self, n):
        pass

    def run_streamed(self, n, chunk, on_rows):
        pass

    def finished(self):
        return []

    def retire(self, slot):
        return np.zeros((0, 2))


def test_pool_executor_runs_fused_cycles_only_with_few_jobs(monkeypatch):
    import torch
    import paper_2105_08026_amd as hbm
    from paper_2105_08026_amd.serve import PoolExecutor
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    pool = _ModePool()
    ex = PoolExecutor(pool, make_workload=None, chunk=8, fused_up_to=2)
    jobs = [Job(j, 0.0, j, 1000, 100) for j in range(3)]
    ex.admit(jobs[0], None)
    ex.run()
    assert pool.modes == [hbm.HBM_CYCLES_FUSED]
    ex.run()                                   # unchanged: no new mode
    assert pool.modes == [hbm.HBM_CYCLES_FUSED]
    ex.admit(jobs[1], None)
    ex.admit(jobs[2], None)
    ex.run()                                   # three resident: two-kernel cycles
    assert pool.modes[-1] == hbm.HBM_CYCLES_GRAPH and len(pool.modes) == 2
    ex.retire(1)
    ex.retire(2)
    ex.run()
    assert pool.modes[-1] == hbm.HBM_CYCLES_FUSED and len(pool.modes) == 3
    # a streamed executor keeps the two-kernel cycle
    pool2 = _ModePool()
    ex2 = PoolExecutor(pool2, make_workload=None, chunk=8, fused_up_to=4, on_rows=lambda *a: None)
    ex2.admit(jobs[0], None)
    ex2.run()
    assert ex2.fused_up_to == 0 and pool2.modes == [hbm.HBM_CYCLES_GRAPH]
