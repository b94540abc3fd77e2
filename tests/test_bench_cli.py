"""bench.py's command line on the host: asking for more than one GPU ends with
a message and a non-zero status before any device work, and the measured
traffic summaries it reads match the current kernel sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_counter_summaries_match_the_kernel_sources():
    import bench
    for workload, n, kind in (("gamma_lf_1d", 300000, "sweep"), ("gamma_lf_1d", 300000, "fused"),
                              ("gamma_lf_color_3d", 1000000, "sweep")):
        t = bench.measured_traffic(workload, n, kind)
        assert t is not None, (workload, n, kind)
        # counted bytes within a few percent of the algorithmic bytes
        alg = bench.BYTES_PER_UPDATE[workload] * n
        assert 0.95 < t["bytes_per_launch"] / alg < 1.2, (workload, t)
