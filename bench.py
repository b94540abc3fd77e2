"""Throughput of the Metropolis-within-Gibbs hot path on one MI355X.

A step is one full cycle of the sampler, by default on the 300,000-object
flux-limited gamma luminosity-function catalog (--workload selects the 3-D
colour catalog at 1,000,000 objects or the normal-normal models): the RAM
sweep of every latent
(Philox draws, proposal, target evaluation, accept, RAM factor update), the
FP64 population log-likelihood reductions, the selection quadrature for the
pending proposal, and the theta Metropolis-Hastings step.  Inputs are
resident in HBM before timing starts.

Prints one JSON line.  value = latent RAM updates per second (N x steps /
wall time); Gibbs sweeps per second are reported alongside.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Kernel arguments of plain launches in device memory (read by the HIP runtime
# at its initialisation, before torch is imported).  The graph-replayed cycles
# of the figure of merit run at the same speed either way; the event-timed
# plain launches that give the sweep kernel's duration otherwise start with a
# read of their arguments from host memory (about 0.8 us longer at N = 3e5).
os.environ.setdefault("HIP_FORCE_DEV_KERNARG", "1")

METRIC = "latent RAM updates/sec and Gibbs sweeps/sec at N=3e5; batched jobs/hour; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per object-update of the sweep: read the latent, RAM
# factor, accept counter and derived data words, write latent, factor and
# counter.  1-D LF (FP32): 4+4+4+12 read, 12 written; 3-D LF (FP32):
# 12+24+4+24 read, 40 written; 1-D normal-normal (FP64): 8+8+4+16 read, 20
# written; 3-D normal-normal (FP64): 24+48+4+24 read, 76 written.
BYTES_PER_UPDATE = {"gamma_lf_1d": 36, "normal_normal_1d": 56, "gamma_lf_color_3d": 104, "normal_normal_3d": 176,
                    "bb1_lf": 36}
# The same per-object state traffic as first planned: the latent, factor, a
# cached log-likelihood and the accept counter read and written, plus the
# data words read (FP32: 1-D 40 B, 3-D 100 B).  The kernels keep no cached
# log-likelihood and read derived data instead, hence BYTES_PER_UPDATE.
PLANNED_BYTES_PER_UPDATE = {"gamma_lf_1d": 40, "gamma_lf_color_3d": 100, "bb1_lf": 40}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="gamma_lf_1d",
                    choices=["gamma_lf_1d", "gamma_lf_color_3d", "normal_normal_1d", "normal_normal_3d",
                             "bb1_lf", "gamma_lf_batch256", "serving", "marginal_gamma_lf_1d", "marginal_bb1_lf",
                             "marginal_normal_normal_1d", "streaming_gamma_lf_1d"])
    ap.add_argument("--horizon", type=float, default=60.0, help="serving: seconds of Poisson arrivals")
    ap.add_argument("--serve-fused-up-to", type=int, default=4,
                    help="serving: fused cycles while at most this many jobs are resident (0: never)")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: arrivals per second")
    ap.add_argument("--sat-jobs", type=int, default=200, help="serving: jobs in the saturation run")
    ap.add_argument("--seq-steps", type=int, default=200,
                    help="batch workload: cycles timed per dataset in the one-dataset-per-launch comparison "
                         "(0 skips it)")
    ap.add_argument("--job-sweeps", type=int, default=2000, help="batch workload: sweeps that make one job")
    ap.add_argument("--n", type=int, default=None,
                    help="objects (default: 300,000; 1,000,000 for the 3-D catalog; 100,000 for BB1)")
    ap.add_argument("--no-graph", action="store_true", help="plain launches (sweep + epilogue kernel per cycle)")
    ap.add_argument("--graph-cycles", action="store_true",
                    help="graph replays of the two-kernel cycle instead of the persistent launch")
    ap.add_argument("--fused-cycles", action="store_true",
                    help="graph replays of fused cycles (one launch per cycle) with the given --launch-shape")
    ap.add_argument("--launch-shape", default="auto", choices=["auto", "1", "2", "4"],
                    help="tiles per sweep workgroup; auto runs the autotuner during burn-in")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 20 times (calibration run for HBM counters)")
    ap.add_argument("--theta-substeps", type=int, default=0,
                    help="single-catalog workloads: 0 for one theta step per cycle from the N-term sums, K >= 1 "
                         "for K steps per cycle from sufficient statistics")
    ap.add_argument("--thin", type=int, default=10, help="streaming: a latent snapshot every THIN sweeps")
    ap.add_argument("--chunk", type=int, default=320, help="streaming: cycles per streamed chunk")
    ap.add_argument("--thetas", type=int, default=64,
                    help="marginal workloads: theta rows evaluated per call (one step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side-c2", action="store_true",
                    help="skip the short 3-D colour catalog run (N = 10^6) reported beside the default workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


KERNEL_SOURCES = ("device.h", "models.h", "kernels.h", "cycles.h")


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2105_08026_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, n: int, kernel: str = "sweep"):
    """HBM bytes per cycle of the sweep kernel (kernel="sweep", one cycle per
    launch) or of the persistent cycle kernel (kernel="cycles") from the
    committed rocprofv3 counter summary for this workload, or None when the
    summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_n{n}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("| ") and line.count("|") == 3:
                key, val = [c.strip() for c in line.strip().strip("|").split("|")]
                vals[key] = val
    if vals.get("kernel_source_digest") != kernel_source_digest():
        return None
    per = float(vals.get("cycles_per_launch", 1))
    fetch = float(vals["fetch_bytes_per_launch"]) / float(vals["copy_fetch_scale"]) / per
    write = float(vals["write_bytes_per_launch"]) / float(vals["copy_write_scale"]) / per
    out = {"bytes_per_launch": fetch + write, "source": os.path.relpath(path, ROOT)}
    if "valu_wave_instructions_per_launch" in vals:
        out["valu_wave_instructions"] = float(vals["valu_wave_instructions_per_launch"]) / per
    return out


# VALU issue capacity: each of the 1024 SIMDs (256 CUs x 4) issues one wave64
# instruction every 4 cycles (16 lanes per cycle) at 2.4 GHz, i.e. 64 lane
# operations per CU per cycle.
SIMDS, VALU_CYCLES_PER_WAVE_INSTR, CLOCK_HZ = 1024, 4, 2.4e9
VALU_PEAK_TOPS = 256 * 64 * CLOCK_HZ / 1e12


def valu_roof(traffic, kern_ms):
    """VALU issue figures of the sweep kernel from the counter summary's
    SQ_INSTS_VALU, or None without one."""
    if not traffic or "valu_wave_instructions" not in traffic or not kern_ms:
        return None
    wi = traffic["valu_wave_instructions"]
    t_issue = wi * VALU_CYCLES_PER_WAVE_INSTR / (SIMDS * CLOCK_HZ)
    achieved = wi * 64 / (kern_ms * 1e-3) / 1e12
    return {"wave_instructions_per_launch": wi, "issue_time_us": 1e6 * t_issue,
            "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "T lane-instructions/s",
            "frac": achieved / VALU_PEAK_TOPS}


def tune_table(hbm, us):
    """The autotuner's microseconds per cycle by candidate (None: not timed)."""
    if us is None:
        return None
    return {k: (None if not np.isfinite(v) else float(v)) for k, v in zip(hbm.tune_labels(), us)}


def planned_frac(name: str, n: int, kern_ms: float) -> dict:
    """The roofline fraction with the planned per-object bytes (PLANNED_BYTES_PER_UPDATE)."""
    pb = PLANNED_BYTES_PER_UPDATE.get(name)
    if not pb or not kern_ms:
        return {}
    gbs = pb * n / (kern_ms * 1e-3) / 1e9
    return {"planned_bytes_per_update": pb, "achieved_planned_bytes": gbs, "frac_planned_bytes": gbs / HBM_PEAK_GBS}


def side_c2(torch, synth, hbm, n: int = 1_000_000, cycles: int = 64):
    """The 3-D colour catalog at N = 10^6, briefly: cycles per second in the
    issue mode the autotuner picks (two-kernel graphs, fused graphs or the
    persistent launch), two-kernel graph replay beside it, and the sweep
    kernel's mean duration (HIP events on its stream, plain launches) with
    its fraction of HBM peak."""
    wl = synth.gamma_lf_3d(n=n)
    s = hbm.Sampler(wl, device="cuda:0", max_cycles=hbm.autotune_cycles(32) + 32 + 4 * cycles)
    pick, tuned = s.autotune(32)
    s.run_cycles(32)
    s.prepare_cycles(cycles)
    torch.cuda.synchronize()
    lc0 = s.launch_counts()
    t0 = time.perf_counter()
    s.run_cycles(cycles)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lc1 = s.launch_counts()
    mode = ("persistent" if lc1["persistent_cycles"] > lc0["persistent_cycles"]
            else "fused graphs" if pick.get("fused") else "two-kernel graphs")
    s.set_cycle_mode(hbm.HBM_CYCLES_GRAPH)
    s.prepare_cycles(cycles)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.run_cycles(cycles)
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t1
    hbm.kernel_timing(s.ctx, True)
    s.run_cycles(cycles, use_graph=False)
    n_launch, kern_ms = hbm.read_kernel_timing(s.ctx)
    hbm.kernel_timing(s.ctx, False)
    assert np.all(np.isfinite(s.theta_trace()))
    s.close()
    bpu = BYTES_PER_UPDATE[wl.name]
    gbs = bpu * n / (kern_ms * 1e-3) / 1e9
    # counted HBM bytes from the committed counter summary of this sweep kernel
    # (one tile per workgroup), over the same event-timed duration
    traffic = measured_traffic(wl.name, n)
    return {"workload": wl.name, "n_objects": n, "cycles_timed": cycles, "us_per_cycle": 1e6 * wall / cycles,
            "issue_mode": mode, "us_per_cycle_two_kernel_graph_replay": 1e6 * wall_graph / cycles,
            "updates_per_s": n * cycles / wall, "tiles_per_workgroup": pick["tiles_per_group"],
            "groups_per_cu_cap": pick["groups_per_cu"], "autotune_us_per_cycle": tune_table(hbm, tuned),
            "sweep_kernel_us": 1e3 * kern_ms, "launches_timed": n_launch, "bytes_per_update": bpu,
            "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
            "traffic_GBps": (traffic["bytes_per_launch"] / (kern_ms * 1e-3) / 1e9) if traffic else None,
            "traffic_bytes_per_launch": traffic["bytes_per_launch"] if traffic else None,
            "traffic_source": traffic["source"] if traffic else "no counter summary for the current kernel sources",
            **planned_frac(wl.name, n, kern_ms)}


def accuracy_vs_oracle(wl, s, o):
    """Errors of this run's FP32/FP64 results against the FP64 oracle, evaluated
    at the GPU's own points: one more (traced) sweep at the current theta gives
    log pi_i at X and at the proposal Y for every object; then the population
    log-likelihood at the resulting latents."""
    theta, _, _ = s.theta()
    chi0 = s.state()[0]
    tr = s.trace_sweep()
    lx = o.log_post(theta, chi0)
    ly = o.log_post(theta, tr[3:3 + wl.d])
    fin = np.isfinite(ly) & np.isfinite(tr[1])
    rel_x = np.abs(tr[0] - lx) / np.maximum(1.0, np.abs(lx))
    rel_y = np.abs(tr[1][fin] - ly[fin]) / np.maximum(1.0, np.abs(ly[fin]))
    chi1 = s.state()[0]
    pl = s.pop_loglik(theta)
    ref = o.pop_loglik(theta, chi1)
    scale = float(np.sum(np.abs(o.pop_terms(theta, chi1))))
    return {"objects": wl.n, "log_density_max_rel_err": float(max(rel_x.max(), rel_y.max())),
            "log_density_median_rel_err": float(np.median(np.concatenate([rel_x, rel_y]))),
            "pop_loglik_abs_err": abs(pl - ref), "pop_loglik_err_rel_to_sum_abs_terms": abs(pl - ref) / scale,
            "theta": theta.tolist()}


def host_cpu() -> dict:
    """The host's CPU model and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "logical_cpus_usable": usable}


def cpu_baseline(wl, seconds: float, sampler=None):
    """The oracle as it stands, timed on the host on a bounded sample of the
    workload (and, given the GPU sampler, the accuracy of its results)."""
    import oracle

    oracle.build(force=False)
    o = oracle.Oracle(wl)
    acc = accuracy_vs_oracle(wl, sampler, o) if sampler is not None else None
    st = o.initial_state()
    o.run(st, 2)                                  # first touch of the arrays
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.run(st, 5)
        done += 5
    dt = time.perf_counter() - t0
    out = {"value": wl.n * done / dt, "unit": "updates/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{done} full MWG cycles of the N={wl.n} catalog ({dt:.1f} s, FP64, OpenMP over objects)",
           "host": host_cpu()}
    # the same on one core, for a quarter of the time
    cores = oracle.num_threads()
    oracle.set_num_threads(1)
    done1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < seconds / 4:
        o.run(st, 1)
        done1 += 1
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    out["one_core"] = {"value": wl.n * done1 / dt1, "unit": "updates/s", "cycles": done1, "seconds": dt1}
    return out, acc


def cpu_baseline_batch(wls, seconds: float):
    """The oracle on the batch's datasets in turn, for a bounded time."""
    import oracle

    oracle.build(force=False)
    done_updates, done_cycles, used, t0 = 0, 0, 0, time.perf_counter()
    for wl in wls:
        if time.perf_counter() - t0 >= seconds:
            break
        o = oracle.Oracle(wl)
        st = o.initial_state()
        o.run(st, 20)
        done_updates += 20 * wl.n
        done_cycles += 20
        used += 1
    dt = time.perf_counter() - t0
    return {"value": done_updates / dt, "unit": "updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"20 full MWG cycles of each of the first {used} datasets ({dt:.1f} s incl. setup, FP64)",
            "host": host_cpu()}


def bench_batch(args, torch, synth, hbm):
    """256 luminosity-function datasets of uneven N advanced together, against
    the same datasets run one per launch sequence."""
    wls = synth.gamma_lf_batch(256)
    n_tot = sum(w.n for w in wls)
    trial = 64
    total = hbm.autotune_cycles(trial) + args.warmup + 2 * args.steps
    b = hbm.Batch(wls, device="cuda:0", max_cycles=total)
    use_graph = not args.no_graph
    if args.launch_shape == "auto":
        pick, us = b.autotune(trial)
    else:
        pick, us = {"tiles_per_group": int(args.launch_shape), "groups_per_cu": 0, "persistent": False}, None
        b.set_launch(pick["tiles_per_group"])
    b.run_cycles(args.warmup, use_graph=use_graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run_cycles(args.steps, use_graph=use_graph)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hbm.kernel_timing(b.ctx, True)
    b.run_cycles(args.steps, use_graph=False)
    n_launch, kern_ms = hbm.read_kernel_timing(b.ctx)
    hbm.kernel_timing(b.ctx, False)
    th_last = [b.theta_trace(j)[-1] for j in (0, 255)]
    assert all(np.all(np.isfinite(t)) for t in th_last)
    b.close()
    del b
    torch.cuda.empty_cache()

    # one dataset per launch sequence: the same datasets, each alone, back to back
    # (skipped with --seq-steps 0)
    seq = 0.0
    for wl in (wls if args.seq_steps > 0 else []):
        s = hbm.Sampler(wl, device="cuda:0", max_cycles=32 + args.seq_steps)
        s.run_cycles(32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.run_cycles(args.seq_steps)
        torch.cuda.synchronize()
        seq += (time.perf_counter() - t1) / args.seq_steps
        s.close()
    t_cycle = wall / args.steps
    jobs_h = 256 * 3600.0 / (args.job_sweeps * t_cycle)
    jobs_h_seq = 256 * 3600.0 / (args.job_sweeps * seq) if seq > 0 else None
    bpu = BYTES_PER_UPDATE["gamma_lf_1d"]
    achieved = bpu * n_tot / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    traffic = measured_traffic("gamma_lf_batch256", n_tot)
    valu = valu_roof(traffic, kern_ms)
    hbm_roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": (traffic["bytes_per_launch"] / (kern_ms * 1e-3) / 1e9) if traffic else None,
                "traffic_bytes_per_launch": traffic["bytes_per_launch"] if traffic else None,
                "algorithmic_bytes_per_launch": bpu * n_tot, "bytes_per_update": bpu}
    if valu is not None:
        # the sweep issues VALU instructions at the SIMDs' rate: that is its roof
        roof = {"bound": "alu", "achieved": valu["achieved"], "peak": valu["peak"], "unit": valu["unit"],
                "frac": valu["frac"], "traffic": hbm_roof["traffic"], "valu": valu, "hbm": hbm_roof}
    else:
        roof = dict(hbm_roof, traffic_source="no counter summary for the current kernel sources")
    roof.update({"kernel": "sweep_kernel<gamma_lf_1d, dataset table>", "launches_timed": n_launch,
                 "kernel_ms": kern_ms})
    out = {
        "metric": METRIC, "value": n_tot * args.steps / wall, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_cycle, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (256 seeded gamma-LF catalogs, N log-uniform on [1e3, 1e5])",
        "config": {"workload": "gamma_lf_batch256", "n_datasets": 256, "n_objects_total": n_tot,
                   "job_sweeps": args.job_sweeps, "graph": use_graph,
                   "tiles_per_workgroup": pick["tiles_per_group"], "groups_per_cu_cap": pick["groups_per_cu"]},
        "jobs_per_hour": jobs_h, "sequential_jobs_per_hour": jobs_h_seq,
        "batch_speedup": jobs_h / jobs_h_seq if jobs_h_seq else None,
        "sequential_ms_per_cycle_sum": 1e3 * seq if seq > 0 else None,
        "autotune_us_per_cycle": tune_table(hbm, us),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(wls, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_serving(args, torch, synth, hbm):
    """Poisson arrivals of luminosity-function jobs served by continuous batching.

    Three runs on one pool: (1) real-time arrivals at --rate for --horizon s
    (latency percentiles), (2) a saturation run with --sat-jobs jobs present
    at t = 0 (capacity in jobs/hour), (3) the saturation jobs one after
    another, each alone in its own context (the one-job-per-launch sampler),
    whose theta traces must equal those from the mix bit for bit.
    """
    from paper_2105_08026_amd import serve as sv

    fth = synth.calibrate_threshold(np.random.default_rng(1), 0.7, 5e10, 4000.0, 0.3)

    def make(job):
        return synth.gamma_lf_1d(n=job.n, seed=job.seed, fth=fth)

    def jobs_of(arr):
        return [sv.Job(i, t, seed, n, sw) for i, (t, seed, n, sw) in enumerate(arr)]

    pool = hbm.Pool(hbm.HBM_GAMMA_LF_1D, capacity=1 << 22, n_slots=128, max_cycles=5000, device="cuda:0")
    ex = sv.PoolExecutor(pool, make, chunk=32, fused_up_to=args.serve_fused_up_to)
    # warm-up: graph capture and first-touch of the pool
    sv.serve(jobs_of([(0.0, 1, 2000, 64), (0.0, 2, 50000, 96)]), ex, prefetch=False)

    live = jobs_of(synth.serving_arrivals(rate=args.rate, horizon_s=args.horizon, seed=4))

    def report(done, total, t):
        print(f"poisson: {done}/{total} jobs done after {t:.0f} s", file=sys.stderr, flush=True)
    res = sv.serve(live, ex, progress=report)
    print(f"poisson: {len(live)} jobs, p50 {res['p50_s']*1e3:.1f} ms, p99 {res['p99_s']*1e3:.1f} ms, "
          f"mean resident {res['mean_resident']:.2f}", file=sys.stderr, flush=True)

    sat_src = synth.serving_arrivals(rate=1e6, horizon_s=1.0, seed=7, job_seed0=50000)[:args.sat_jobs]
    sat = jobs_of([(0.0, seed, n, sw) for _, seed, n, sw in sat_src])
    wls = {j.id: make(j) for j in sat}
    res_sat = sv.serve(sat, ex, make=lambda j: wls[j.id], prefetch=False)
    print(f"saturation: {len(sat)} jobs in {res_sat['wall_s']:.2f} s, mean resident {res_sat['mean_resident']:.1f}",
          file=sys.stderr, flush=True)
    pool.close()

    seq, same = 0.0, 0
    traces = {j.id: j.trace for j in res_sat["jobs"]}
    for j in sat:
        s = hbm.Sampler(wls[j.id], device="cuda:0", max_cycles=j.sweeps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.run_cycles(j.sweeps)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t1
        same += int(np.array_equal(s.theta_trace(), traces[j.id]))
        s.close()
    jph_sat = 3600.0 * len(sat) / res_sat["wall_s"]
    jph_seq = 3600.0 * len(sat) / seq
    out = {
        "metric": METRIC, "value": jph_sat, "unit": "jobs/hour", "n_gpus": 1, "steps": len(sat), "warmup": 2,
        "ms_per_step": 1e3 * res_sat["wall_s"] / len(sat), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded gamma-LF jobs, N log-uniform on [1e3, 3e5], budgets in {1000, 2000, 5000})",
        "config": {"workload": "serving", "rate_per_s": args.rate, "horizon_s": args.horizon,
                   "pool_objects": 1 << 22, "pool_slots": 128, "chunk_cycles": 32,
                   "fused_cycles_up_to_jobs": ex.fused_up_to},
        "poisson": {"jobs": len(live), "p50_s": res["p50_s"], "p99_s": res["p99_s"], "mean_s": res["mean_s"],
                    "jobs_per_hour": res["jobs_per_hour"], "mean_resident": res["mean_resident"],
                    "gpu_busy_frac": res["busy_s"] / res["wall_s"], "wait_for_inputs_s": res["wait_for_inputs_s"]},
        "saturation": {"jobs": len(sat), "wall_s": res_sat["wall_s"], "jobs_per_hour": jph_sat,
                       "p50_s": res_sat["p50_s"], "p99_s": res_sat["p99_s"],
                       "mean_resident": res_sat["mean_resident"]},
        "sequential": {"jobs_per_hour": jph_seq, "wall_s": seq},
        "served_vs_sequential": jph_sat / jph_seq,
        "alone_vs_mix_identical": f"{same}/{len(sat)}",
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


# FP64 operations per object integral of the marginal kernel (an FMA counts
# two): 64 x (ADD + MUL + 2 FMA + TRANS) from the SQ_INSTS_VALU_*_F64
# counters of the marginal bench command, per launch, divided by N x theta
# rows (theta near the truth; the count depends on how many objects need the
# region below the datum).
FLOPS_PER_INTEGRAL = {"marginal_gamma_lf_1d": 8250, "marginal_bb1_lf": 55670, "marginal_normal_normal_1d": 3310}
FP64_PEAK_TFLOPS = 78.6
NODES_PER_OBJECT = {"marginal_gamma_lf_1d": 216, "marginal_bb1_lf": 216, "marginal_normal_normal_1d": 48}


def cpu_baseline_marginal(wl, theta, seconds: float):
    """The oracle's marginal terms, timed on a bounded prefix of the catalog."""
    import copy

    import oracle

    oracle.build(force=False)
    m = min(wl.n, 2000)
    sub = copy.copy(wl)
    sub.data = np.ascontiguousarray(wl.data[:, :m])
    sub.chi0 = np.ascontiguousarray(wl.chi0[:, :m])
    sub.n = m
    o = oracle.Oracle(sub)
    o.marginal_terms(theta)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.marginal_terms(theta)
        done += 1
    dt = time.perf_counter() - t0
    return {"value": m * done / dt, "unit": "object integrals/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} evaluations of the first {m} objects' marginal terms at one theta ({dt:.1f} s, FP64, "
                      "one thread)", "host": host_cpu()}


def bench_marginal(args, torch, synth, hbm):
    """Latent-free log-likelihood of theta, each object's latent integrated out
    by per-object quadrature (Sec. 6).  A step is one call evaluating
    --thetas theta rows over the whole catalog."""
    make = {"marginal_gamma_lf_1d": (synth.gamma_lf_1d, 300_000), "marginal_bb1_lf": (synth.bb1_lf, 100_000),
            "marginal_normal_normal_1d": (synth.normal_normal_1d, 300_000)}
    gen, n_default = make[args.workload]
    wl = gen(n=args.n or n_default)
    s = hbm.Sampler(wl, device="cuda:0", max_cycles=8)
    rng = np.random.default_rng(0)
    th0 = np.array(wl.theta_true, dtype=np.float64)
    ths = th0 + 0.01 * rng.standard_normal((args.thetas, wl.p))
    for _ in range(max(1, args.warmup // 20)):
        s.marginal_loglik(ths)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = s.marginal_loglik(ths)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert np.all(np.isfinite(out)), "non-finite marginal log-likelihood"
    # kernel durations from HIP events on the sampler's stream
    n_ev = min(args.steps, 200)
    hbm.kernel_timing(s.ctx, True)
    for _ in range(n_ev):
        s.marginal_loglik(ths)
    n_launch, kern_ms = hbm.read_kernel_timing(s.ctx)
    hbm.kernel_timing(s.ctx, False)
    # one theta per call: the rate a Metropolis chain on theta would step at
    n_one = 1000
    t1 = time.perf_counter()
    for j in range(n_one):
        s.marginal_loglik(ths[j % args.thetas])
    one_wall = time.perf_counter() - t1
    hbm.kernel_timing(s.ctx, True)
    for j in range(200):
        s.marginal_loglik(ths[j % args.thetas])
    _, kern_one_ms = hbm.read_kernel_timing(s.ctx)
    hbm.kernel_timing(s.ctx, False)
    nodes = NODES_PER_OBJECT[args.workload] * wl.n * args.thetas
    fpi = FLOPS_PER_INTEGRAL[args.workload]
    achieved = fpi * wl.n * args.thetas / (kern_ms * 1e-3) / 1e12 if (fpi and kern_ms > 0) else None
    out = {
        "metric": METRIC, "value": wl.n * args.thetas * args.steps / wall, "unit": "object integrals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": f"synthetic (seeded {wl.name} catalog; theta rows near the truth)",
        "config": {"workload": args.workload, "n_objects": wl.n, "thetas_per_step": args.thetas,
                   "nodes_per_object": NODES_PER_OBJECT[args.workload]},
        "theta_evaluations_per_s": args.thetas * args.steps / wall,
        "single_theta": {"calls_per_s": n_one / one_wall, "ms_per_call": 1e3 * one_wall / n_one,
                         "kernel_ms": kern_one_ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS if achieved else None, "traffic": None,
                     "kernel": f"marginal_kernel<{wl.name}>", "flops_per_object_integral": fpi,
                     "nominal_node_evaluations": nodes,
                     "kernel_ms": kern_ms, "launches_timed": n_launch},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_marginal(wl, th0, args.cpu_seconds)
    s.close()
    print(json.dumps(out), flush=True)


def bench_streaming(args, torch, synth, hbm):
    """Latent snapshots every --thin sweeps of the 300,000-object gamma-LF
    catalog, streamed to the host through a ring of 2 ceil(chunk / thin)
    device rows, against the same cycles with no snapshots and with every
    snapshot kept in a full device buffer."""
    import os
    import tempfile

    wl = synth.gamma_lf_1d(n=args.n or 300_000)
    steps, thin, chunk = args.steps, args.thin, args.chunk
    ring = 2 * (-(-chunk // thin))
    row_bytes = wl.n * 4

    def timed(s, run):
        s.run_cycles(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    total = args.warmup + steps
    plain = hbm.Sampler(wl, device="cuda:0", max_cycles=total)
    plain.set_launch(1)
    t_plain = timed(plain, lambda: plain.run_cycles(steps))
    plain.close()
    full = hbm.Sampler(wl, device="cuda:0", max_cycles=total, thin=thin)
    full.set_launch(1)
    t_full = timed(full, lambda: full.run_cycles(steps))
    full_rows = full.snaps.shape[0]
    full.close()
    del full
    torch.cuda.empty_cache()
    got = {"rows": 0}

    def count(first, rows):
        got["rows"] += rows.shape[0]
        return False
    st = hbm.Sampler(wl, device="cuda:0", max_cycles=total, thin=thin, snap_rows=ring)
    st.set_launch(1)
    t_stream = timed(st, lambda: st.run_streamed(steps, chunk, count, copy=False))
    st.close()
    hr = hbm.Sampler(wl, device="cuda:0", max_cycles=total, thin=thin, snap_rows=ring, snap_host=True)
    hr.set_launch(1)
    got_h = {"rows": 0}

    def count_h(first, rows):
        got_h["rows"] += rows.shape[0]
        return False
    t_hring = timed(hr, lambda: hr.run_streamed(steps, chunk, count_h, copy=False))
    hr.close()
    fs = hbm.Sampler(wl, device="cuda:0", max_cycles=total, thin=thin, snap_rows=ring)
    fs.set_launch(1)
    fd, path = tempfile.mkstemp(dir=os.environ.get("TMPDIR", "/tmp"), suffix=".f32")
    os.close(fd)
    try:
        t_file = timed(fs, lambda: fs.run_to_file(steps, chunk, path))
        file_bytes = os.path.getsize(path)
    finally:
        os.unlink(path)
    fs.close()
    rows_streamed = (args.warmup + steps) // thin - args.warmup // thin
    out = {
        "metric": METRIC, "value": wl.n * steps / t_stream, "unit": "updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_stream / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded gamma_lf_1d catalog)",
        "config": {"workload": "streaming_gamma_lf_1d", "n_objects": wl.n, "thin": thin, "chunk_cycles": chunk,
                   "ring_rows": ring},
        "us_per_cycle": {"no_snapshots": 1e6 * t_plain / steps, "full_device_buffer": 1e6 * t_full / steps,
                         "streamed_to_host": 1e6 * t_stream / steps, "streamed_to_file": 1e6 * t_file / steps,
                         "host_ring_zero_copy": 1e6 * t_hring / steps},
        "snapshot_device_bytes": {"full_device_buffer": full_rows * row_bytes, "streamed_ring": ring * row_bytes},
        "rows_delivered": got["rows"], "rows_delivered_host_ring": got_h["rows"], "rows_expected": rows_streamed,
        "file_bytes": file_bytes,
        "d2h_GBps_streamed": rows_streamed * row_bytes / t_stream / 1e9,
        "d2h_GBps_host_ring": rows_streamed * row_bytes / t_hring / 1e9,
        "d2h_GBps_to_file": rows_streamed * row_bytes / t_file / 1e9,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding a catalog's objects over "
              "several GPUs (one all-gather of tile partials per cycle) is a design, not launched here",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    import paper_2105_08026_amd as hbm

    torch.cuda.set_device(0)
    if args.copy_probe:
        # a plain device-to-device copy of known size: the reference for scaling
        # the FETCH_SIZE / WRITE_SIZE counters of the sampler's kernels
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 20}), flush=True)
        return
    if args.workload == "gamma_lf_batch256":
        bench_batch(args, torch, synth, hbm)
        return
    if args.workload == "serving":
        bench_serving(args, torch, synth, hbm)
        return
    if args.workload.startswith("marginal_"):
        bench_marginal(args, torch, synth, hbm)
        return
    if args.workload == "streaming_gamma_lf_1d":
        bench_streaming(args, torch, synth, hbm)
        return
    make = {"gamma_lf_1d": (synth.gamma_lf_1d, 300_000), "gamma_lf_color_3d": (synth.gamma_lf_3d, 1_000_000),
            "normal_normal_1d": (synth.normal_normal_1d, 300_000), "normal_normal_3d": (synth.normal_normal_3d, 300_000),
            "bb1_lf": (synth.bb1_lf, 100_000)}
    gen, n_default = make[args.workload]
    wl = gen(n=args.n or n_default)
    trial = 64
    total = hbm.autotune_cycles(trial) + args.warmup + 4 * args.steps
    s = hbm.Sampler(wl, device="cuda:0", max_cycles=total, theta_substeps=args.theta_substeps)
    use_graph = not args.no_graph
    if args.graph_cycles:
        s.set_cycle_mode(hbm.HBM_CYCLES_GRAPH)
    if args.fused_cycles:
        s.set_cycle_mode(hbm.HBM_CYCLES_FUSED)

    # burn-in: the launch-shape autotuner's cycles (or a fixed shape), then warm-up cycles
    if args.launch_shape == "auto":
        pick, tuned = s.autotune(trial)
    else:
        pick, tuned = {"tiles_per_group": int(args.launch_shape), "groups_per_cu": 0, "persistent": None,
                       "fused": None}, None
        s.set_launch(pick["tiles_per_group"])
    s.run_cycles(args.warmup, use_graph=use_graph)
    if use_graph:
        s.prepare_cycles(args.steps)          # any graph capture happens outside the timed region
    torch.cuda.synchronize()

    # Timed region 1: the figure of merit -- one persistent launch of all the
    # cycles where the context allows it, else graph replays.
    lc0 = s.launch_counts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run_cycles(args.steps, use_graph=use_graph)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lc1 = s.launch_counts()
    issued = {key: lc1[key] - lc0[key] for key in lc0}
    assert issued["replayed_cycles"] + issued["plain_cycles"] + issued["persistent_cycles"] == args.steps, issued
    persistent = issued["persistent_launches"] > 0
    fused = bool(pick.get("fused") or args.fused_cycles) and issued["replayed_cycles"] == args.steps

    # Timed region 2: the same way of issuing, each launch bracketed by HIP
    # events on the sampler's stream, for the dominant kernel's duration (the
    # persistent kernel; the fused-cycle kernel of plain fused launches; with
    # two-kernel graphs, the sweep kernel of plain launches).
    hbm.kernel_timing(s.ctx, True)
    s.run_cycles(args.steps, use_graph=use_graph)
    n_launch_dom, dom_ms = hbm.read_kernel_timing(s.ctx)
    # Timed region 3: the two-kernel cycle as plain launches, for the sweep
    # kernel's own duration.
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.run_cycles(args.steps, use_graph=False)
    torch.cuda.synchronize()
    wall_ev = time.perf_counter() - t1
    n_launch, kern_ms = hbm.read_kernel_timing(s.ctx)
    hbm.kernel_timing(s.ctx, False)
    # The two-kernel cycle replayed from graphs, for comparison.
    mode_graph = None
    if persistent or fused:
        s.set_cycle_mode(hbm.HBM_CYCLES_GRAPH)
        s.prepare_cycles(args.steps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.run_cycles(args.steps)
        torch.cuda.synchronize()
        mode_graph = time.perf_counter() - t2
        s.set_cycle_mode(hbm.HBM_CYCLES_FUSED if fused else hbm.HBM_CYCLES_AUTO)

    th = s.theta_trace()
    assert np.all(np.isfinite(th)), "non-finite theta"
    stats = s.stats()
    # effective samples of theta per second over the cycles of timed region 1
    i_fom = hbm.autotune_cycles(trial) + args.warmup if args.launch_shape == "auto" else args.warmup
    tw = th[i_fom:i_fom + args.steps]
    ess = []
    for j in range(wl.p):
        b = max(2, int(np.sqrt(len(tw))))
        xb = tw[: b * (len(tw) // b), j].reshape(b, -1).mean(axis=1)
        se2 = xb.var(ddof=1) / b
        ess.append(float(tw[:, j].var() / se2) if se2 > 0 else None)

    updates = wl.n * args.steps / wall
    bpu = BYTES_PER_UPDATE[wl.name]
    sweep_gbs = bpu * wl.n / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    sweep_traffic = measured_traffic(wl.name, wl.n, "sweep")
    sweep_roof = {"kernel": f"sweep_kernel<{wl.name}>", "kernel_ms": kern_ms, "launches_timed": n_launch,
                  "achieved": sweep_gbs, "frac": sweep_gbs / HBM_PEAK_GBS if sweep_gbs else None,
                  "traffic": (sweep_traffic["bytes_per_launch"] / (kern_ms * 1e-3) / 1e9) if sweep_traffic else None,
                  "traffic_source": sweep_traffic["source"] if sweep_traffic else
                  "no counter summary for the current kernel sources",
                  "valu": valu_roof(sweep_traffic, kern_ms), **planned_frac(wl.name, wl.n, kern_ms)}
    if persistent:
        # one persistent launch = args.steps cycles = N x steps object-updates
        cyc_ms = dom_ms / args.steps if dom_ms > 0 else 0.0
        achieved = bpu * wl.n / (cyc_ms * 1e-3) / 1e9 if cyc_ms > 0 else None
        traffic = measured_traffic(wl.name, wl.n, "cycles")
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": (traffic["bytes_per_launch"] / (cyc_ms * 1e-3) / 1e9) if traffic else None,
                "traffic_bytes_per_cycle": traffic["bytes_per_launch"] if traffic else None,
                "algorithmic_bytes_per_launch": bpu * wl.n * args.steps, "bytes_per_update": bpu,
                "traffic_source": traffic["source"] if traffic else "no counter summary for the current kernel sources",
                "kernel": f"cycles_kernel<{wl.name}>", "cycles_per_launch": args.steps,
                "launch_ms": dom_ms, "us_per_cycle_in_kernel": 1e3 * cyc_ms, "launches_timed": n_launch_dom,
                "valu": valu_roof(traffic, cyc_ms), **planned_frac(wl.name, wl.n, cyc_ms),
                "sweep_kernel_two_kernel_cycle": sweep_roof}
    elif fused:
        # one fused launch = one cycle: the previous sweep's theta step in every
        # workgroup, then the sweep of N objects
        achieved = bpu * wl.n / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else None
        traffic = measured_traffic(wl.name, wl.n, "fused")
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": (traffic["bytes_per_launch"] / (dom_ms * 1e-3) / 1e9) if traffic else None,
                "traffic_bytes_per_launch": traffic["bytes_per_launch"] if traffic else None,
                "algorithmic_bytes_per_launch": bpu * wl.n, "bytes_per_update": bpu,
                "traffic_source": traffic["source"] if traffic else "no counter summary for the current kernel sources",
                # the kernel the launch shape selects; the committed counters of the
                # fused cycle were taken with two tiles per workgroup
                "kernel": (f"fused_wide_kernel<{wl.name}, {pick['tiles_per_group']}>" if pick["tiles_per_group"] > 1
                           else f"fused_kernel<{wl.name}>"),
                "traffic_counted_with_tiles_per_workgroup": 2,
                "kernel_ms": dom_ms, "launches_timed": n_launch_dom,
                "valu": valu_roof(traffic, dom_ms), **planned_frac(wl.name, wl.n, dom_ms),
                "sweep_kernel_two_kernel_cycle": sweep_roof}
    else:
        roof = {"bound": "hbm", "achieved": sweep_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (sweep_gbs / HBM_PEAK_GBS) if sweep_gbs else None,
                "traffic": sweep_roof["traffic"],
                "traffic_bytes_per_launch": sweep_traffic["bytes_per_launch"] if sweep_traffic else None,
                "algorithmic_bytes_per_launch": bpu * wl.n, "bytes_per_update": bpu,
                "traffic_source": sweep_roof["traffic_source"], "kernel": f"sweep_kernel<{wl.name}>",
                "launches_timed": n_launch, "valu": sweep_roof["valu"], **planned_frac(wl.name, wl.n, kern_ms)}
    out = {
        "metric": METRIC,
        "value": updates,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.precision == "f32" else "f64",
        "data": f"synthetic (seeded {wl.name} catalog)",
        "config": {"workload": wl.name, "n_objects": wl.n, "latent_dim": wl.d, "theta_dim": wl.p,
                   "selection_quadrature_nodes": 512 if wl.model in (2, 3, 5) else 0,
                   "persistent_launch": persistent, "fused_cycles": fused,
                   "graph": issued["graph_replays"] > 0 and issued["plain_cycles"] == 0,
                   "sweeps_per_step": 1, "tiles_per_workgroup": pick["tiles_per_group"],
                   "groups_per_cu_cap": pick["groups_per_cu"], "autotune_picked_persistent": pick["persistent"],
                   "autotune_picked_fused": pick.get("fused"),
                   "theta_substeps": args.theta_substeps},
        "timed_cycles_issued": issued,
        "theta_ess_per_s": [e / wall if e else None for e in ess],
        "autotune_us_per_cycle": tune_table(hbm, tuned),
        "gibbs_sweeps_per_s": args.steps / wall,
        "breakdown_ms": {"step": 1e3 * wall / args.steps, "sweep_kernel": kern_ms,
                         "step_two_kernel_plain_launches_event_timed": 1e3 * wall_ev / args.steps,
                         "step_two_kernel_graph_replay": 1e3 * mode_graph / args.steps if mode_graph else None,
                         "persistent_launch_ms": dom_ms if persistent else None,
                         "fused_kernel": dom_ms if fused else None},
        "roofline": roof,
        "accept_rate_last_sweep": stats["n_acc"] / wl.n,
        "theta_last": th[-1].tolist(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy_vs_oracle"] = cpu_baseline(wl, args.cpu_seconds, sampler=s)
    s.close()
    if wl.name == "gamma_lf_1d" and not args.no_side_c2:
        torch.cuda.empty_cache()
        out["gamma_lf_color_3d_n1000000"] = side_c2(torch, synth, hbm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
