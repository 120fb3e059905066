"""Host-side checks of the benchmark's command line (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The counting path runs on one GPU: --gpus above 1 exits with status 2 and says so
    in one JSON line, before any GPU work."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["requested_gpus"] == 2
    assert "one GPU" in line["error"]


def test_source_hash_is_stable():
    """The hash that ties profiles/hbm_traffic.json to the kernel sources depends only on
    those sources."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.src_hash() == bench.src_hash()
    assert len(bench.src_hash()) == 16
