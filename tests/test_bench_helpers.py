"""Host-side pieces of bench.py: the algorithmic byte counts, the counter
traffic lookup and the one-GPU guard (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_formula():
    # N = 10 triangles, 4 visible, 6 instances, 2x3 image, SH degree 1 (K = 4)
    b = bench.algorithmic_bytes(10, 4, 6, 2, 3, 4)
    sh = 12 * 4
    assert b["project"] == 44 * 10 + sh * 4 + 48 * 4
    assert b["bin_sort"] == 36 * 6
    assert b["raster_fwd"] == 48 * 4 + 4 * 6 + 28 * 6
    assert b["raster_bwd"] == 12 * 6 + 8 * 6 + 4 * 6 + 48 * 4 + 2 * 48 * 4
    assert b["project_bwd"] == (44 + sh) * 4 + 48 * 4 + (44 + sh) * 10


def test_traffic_is_tied_to_the_kernel_source():
    for name, t in bench.TRAFFIC.items():
        got = bench.traffic_bytes(name)
        if t["src"] is None or bench._sha(t["files"]) != t["src"]:
            assert got is None
        else:
            want = 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])
            assert got == want
    assert bench.traffic_bytes("no such kernel") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip())["error"]
