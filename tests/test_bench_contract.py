"""bench.py's contract pieces that need no GPU: one GPU only, the per-entry
flop accounting of the roofline, and the rel-L2 figures it reports."""
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


def test_batch_rel_l2_against_the_oracle(oracle_mod):
    """The batch's accuracy figure: outputs equal to the oracle's give 0, and
    outputs off by a relative 1e-4 give 1e-4 (the back projection is checked
    as the back projection of the batch's own sinograms)."""
    import numpy as np

    import bench
    from paper_1907_10526_amd import phantoms, workloads
    s = workloads.SMALL
    og = oracle_mod.Geometry(**s.kwargs())
    imgs = np.stack([workloads.phantom(s, seed=500 + b) for b in range(3)])
    y = np.stack([og.forward(imgs[b].astype(np.float64)) for b in range(3)])
    z = np.stack([og.back(y[b]) for b in range(3)])
    exact = bench.batch_rel_l2(og, (imgs, y, z))
    assert exact["forward"] <= 1e-12 and exact["back"] <= 1e-12
    fwd_off = bench.batch_rel_l2(og, (imgs, y * (1 + 1e-4), z * (1 + 1e-4)))
    assert abs(fwd_off["forward"] - 1e-4) <= 1e-8 and fwd_off["back"] <= 1e-12
    back_off = bench.batch_rel_l2(og, (imgs, y, z * (1 - 1e-4)))
    assert back_off["forward"] <= 1e-12 and abs(back_off["back"] - 1e-4) <= 1e-8
    assert "3 images" in back_off["sample"]
