"""Host-side checks of bench.py (CPU only).

* one GPU only: --gpus 2 exits with status 2 and a message, before touching torch or a device;
* the committed counter profile (profiles/traffic.json) was taken on the committed kernel sources,
  so the benchmark reports its HBM traffic, and it covers the dominant pass kernel.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_profile_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench

    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert t["kernel_src_sha256_16"] == bench.kernel_hash()
    assert bench.load_traffic("fast_pass<5, false, true, double>") is not None
