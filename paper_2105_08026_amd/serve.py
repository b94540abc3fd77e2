"""Continuous-batching request loop over a pool of resident datasets.

Inference jobs (a catalog plus a sweep budget) arrive over time.  The loop
admits them first come, first served, whenever a slot and a contiguous run
of object tiles are free (admission by memory footprint: a job needs
ceil(N / 256) tiles of the pool's packed buffers), advances every resident
job together in chunks of full sampler cycles (one graph replay covers all
of them), lets the device stop each job exactly at its budget, and retires
finished jobs to free their slot and tiles for the queue.  Chain state stays
in HBM from admission to retirement.

The scheduling logic is independent of the device: an executor provides
fits / admit / run / retire, so the same loop runs over the GPU pool
(:class:`PoolExecutor`) or over a simulated one in tests.
"""

from __future__ import annotations

import collections
import dataclasses
import queue as _queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Job:
    id: int
    arrival: float                 # seconds after the start of the run
    seed: int
    n: int                         # objects
    sweeps: int                    # theta steps (= sweeps) to run
    admitted: Optional[float] = None
    done: Optional[float] = None
    slot: Optional[int] = None
    trace: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class TileAllocator:
    """First-fit allocator of contiguous tile runs; owner -1 marks a free tile."""

    def __init__(self, n_tiles: int):
        self.owner = np.full(n_tiles, -1, dtype=np.int64)

    def find(self, nt: int) -> Optional[int]:
        free = np.concatenate(([False], self.owner < 0, [False]))
        d = np.diff(free.astype(np.int8))
        starts, ends = np.flatnonzero(d == 1), np.flatnonzero(d == -1)
        ok = np.flatnonzero(ends - starts >= nt)
        return int(starts[ok[0]]) if ok.size else None

    def take(self, start: int, nt: int, owner: int):
        assert np.all(self.owner[start:start + nt] < 0), "tiles already taken"
        self.owner[start:start + nt] = owner

    def release(self, owner: int):
        self.owner[self.owner == owner] = -1

    @property
    def free_tiles(self) -> int:
        return int(np.count_nonzero(self.owner < 0))


class PoolExecutor:
    """Runs the loop's decisions on a :class:`paper_2105_08026_amd.Pool`.

    cfg: extra dataset settings for every job (e.g. thin, theta_substeps).
    on_rows(job, first, rows): when given, every chunk is a streamed run and
    each job's latent snapshots reach it as they are taken (the pool then
    needs only snap_rows = 2 ceil(chunk / thin) rows of device memory).
    fused_up_to: chunks run as fused cycles (one launch per cycle, every
    tile's workgroup taking its own job's theta step) while at most this many
    jobs are resident, as two-kernel cycles above (0: always two-kernel).
    With few small jobs the fused cycle is 7-18 % faster; with many, each
    tile's redundant theta step costs more than the launch it saves.  The
    choice changes no result.
    """

    def __init__(self, pool, make_workload: Callable[[Job], object], chunk: int = 32, cfg: Optional[dict] = None,
                 on_rows: Optional[Callable] = None, fused_up_to: int = 4):
        self.pool, self.make, self.chunk = pool, make_workload, chunk
        self.max_tiles = pool.tiles.size
        self.cfg = dict(cfg or {})
        self.on_rows = on_rows
        self.fused_up_to = int(fused_up_to) if on_rows is None else 0
        self.mode = None
        self.jobs = {}

    def fits(self, job: Job) -> bool:
        return self.pool.fits(job.n)

    def too_big(self, job: Job) -> bool:
        return -(-job.n // 256) > self.max_tiles or job.sweeps > self.pool.max_cycles

    def admit(self, job: Job, wl) -> int:
        (slot,) = self.pool.admit([wl], [job.sweeps], **self.cfg)
        assert slot is not None
        self.jobs[slot] = job
        return slot

    def run(self) -> List[int]:
        import torch
        from . import HBM_CYCLES_FUSED, HBM_CYCLES_GRAPH
        mode = HBM_CYCLES_FUSED if len(self.jobs) <= self.fused_up_to else HBM_CYCLES_GRAPH
        if mode != self.mode:
            self.pool.set_cycle_mode(mode)
            self.mode = mode
        if self.on_rows is None:
            self.pool.run_cycles(self.chunk)
        else:
            self.pool.run_streamed(self.chunk, self.chunk,
                                   lambda slot, first, rows: self.on_rows(self.jobs[slot], first, rows))
        torch.cuda.synchronize(self.pool.device)
        return self.pool.finished()

    def retire(self, slot: int) -> np.ndarray:
        self.jobs.pop(slot, None)
        return self.pool.retire(slot)


class _Prefetcher:
    """Builds job inputs ahead of their arrival on a background thread."""

    def __init__(self, jobs: List[Job], make: Callable[[Job], object], depth: int = 64):
        self.q: _queue.Queue = _queue.Queue(maxsize=depth)
        self.t = threading.Thread(target=self._run, args=(jobs, make), daemon=True)
        self.t.start()

    def _run(self, jobs, make):
        for j in jobs:
            self.q.put((j, make(j)))

    def next(self):
        return self.q.get()


def serve(jobs: List[Job], executor, make: Optional[Callable[[Job], object]] = None,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          prefetch: bool = True, progress: Optional[Callable[[int, int, float], None]] = None,
          progress_every_s: float = 30.0) -> dict:
    """Runs the request loop until every job is done; returns the jobs and loop statistics.

    Jobs must be sorted by arrival time.  A job is visible to the loop once
    the clock passes its arrival; its latency is completion minus arrival.
    progress (optional) is called with (jobs finished, jobs, seconds since
    the start) at most every progress_every_s seconds.
    """
    make = make or executor.make
    for j in jobs:
        if executor.too_big(j):
            raise ValueError(f"job {j.id} (N={j.n}, {j.sweeps} sweeps) can never fit the pool")
    src = _Prefetcher(jobs, make) if prefetch else None
    t0 = clock()
    nxt = 0
    ready = collections.deque()          # arrived, waiting for admission: (job, workload)
    resident = {}
    finished: List[Job] = []
    busy = 0.0
    chunks = 0
    resident_sum = 0
    wait_gen = 0.0
    last_report = 0.0
    while len(finished) < len(jobs):
        now = clock() - t0
        if progress is not None and now - last_report >= progress_every_s:
            progress(len(finished), len(jobs), now)
            last_report = now
        while nxt < len(jobs) and jobs[nxt].arrival <= now:
            if src is not None:
                tg = clock()
                job, wl = src.next()
                wait_gen += clock() - tg
            else:
                job, wl = jobs[nxt], make(jobs[nxt])
            assert job is jobs[nxt]
            ready.append((job, wl))
            nxt += 1
        # first come, first served: admit from the head while it fits
        while ready and executor.fits(ready[0][0]):
            job, wl = ready.popleft()
            job.slot = executor.admit(job, wl)
            job.admitted = clock() - t0
            resident[job.slot] = job
        if resident:
            tb = clock()
            done_slots = executor.run()
            busy += clock() - tb
            chunks += 1
            resident_sum += len(resident)
            t_done = clock() - t0
            for slot in done_slots:
                job = resident.pop(slot)
                job.trace = executor.retire(slot)
                job.done = t_done
                finished.append(job)
        elif nxt < len(jobs):
            sleep(max(0.0, jobs[nxt].arrival - (clock() - t0)))
        else:
            raise RuntimeError("jobs waiting but nothing resident and nothing arriving")
    wall = clock() - t0
    lat = np.array([j.latency for j in finished])
    return {
        "jobs": finished, "wall_s": wall, "busy_s": busy, "chunks": chunks,
        "mean_resident": resident_sum / max(chunks, 1), "wait_for_inputs_s": wait_gen,
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()), "jobs_per_hour": 3600.0 * len(finished) / wall,
    }
