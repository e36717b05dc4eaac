"""Host-side checks of bench.py (no GPU needed)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_is_read_for_its_own_digest_only():
    path = os.path.join(ROOT, "profiles", "traffic_channel_1M.txt")
    lines = open(path).read().splitlines()
    digest = next(l.split(":", 1)[1].strip() for l in lines if l.startswith("source_digest:"))
    shape = next(l for l in lines if l.startswith("shape: k_iter")).split(":", 1)[1].split()
    launch = {"iter_shape": int(shape[1]), "tile_rows": int(shape[2]), "block": int(shape[3])}
    got = bench.measured_traffic("channel_1M", launch, "k_iter")
    if digest == bench.source_digest():
        assert got == float(shape[4])
    else:
        assert got is None  # the kernels changed since the counters were taken
    assert bench.measured_traffic("channel_1M", {"iter_shape": 9, "tile_rows": 1, "block": 1},
                                  "k_iter") is None
    assert bench.measured_traffic("no_such_workload", launch, "k_iter") is None
