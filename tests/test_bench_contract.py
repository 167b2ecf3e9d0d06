"""bench.py contract pieces that run without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_measured_traffic_lookup_requires_matching_sources():
    sys.path.insert(0, ROOT)
    import bench
    # a configuration with no committed counter summary has no traffic figure
    assert bench.measured_traffic("jitter7_p9", "f64", 1, (13,), 1) is None
