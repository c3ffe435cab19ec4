"""bench.py's contract pieces that need no GPU: one GPU only, and the
per-entry flop accounting of the roofline."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_flops_per_entry():
    import bench
    assert bench.FLOPS_PER_ENTRY == 48
    assert bench.flops_per_entry(1) == 48
    assert bench.flops_per_entry(4) == 13.5
    assert bench.flops_per_entry(8) == 7.75
