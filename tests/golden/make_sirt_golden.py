"""Write the stored SIRT reference values used by the GPU parity tests.

Every stored value is computed by the FP64 oracle (``oracle/``) from seeded
inputs (``paper_1907_10526_amd.phantoms``); nothing comes from the GPU
library.  Run from the repository root:

    python tests/golden/make_sirt_golden.py [--skip-large]

Outputs (numpy ``.npz``, no pickled objects):

* ``sirt50_reduced.npz``: the 50-step SIRT iterate, from zero, on a 256 x 256
  scan with the large scan's proportions (180 views over 2 pi, 256 cells of
  width 1, source-centre 500, source-detector 750).  The data are Poisson
  counts (I0 = 1e5, seed 33) of a non-negative 20-ellipse phantom (seed 3)
  scaled so that the largest line integral is 4.
* ``sirt2_large_sampled.npz``: pixels of the second SIRT iterate, from zero,
  on the full 2048 x 2048, 1440-view, 2048-cell scan (source-centre 4000,
  source-detector 6000) with a seeded uniform U[0, 4] sinogram (seed 77), at
  256 seeded pixel positions (seed 78).  Two steps need the row sums, the
  column sums, two back projections and one forward projection at full size
  (about 10-20 minutes of FP64 CPU work).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1907_10526_amd import phantoms, workloads  # noqa: E402

REDUCED = workloads.Scan("sirt-reduced", 256, 180, 256, 1.0, 500.0, 750.0)


def reduced_inputs():
    """Phantom, clean and noisy sinograms of the reduced SIRT workload."""
    s = REDUCED
    scale = s.n / 64.0
    c = np.clip(phantoms.ellipses(s.n, 20, 3, (4.0 * scale, 20.0 * scale)).astype(np.float64), 0.0, None)
    og = oracle.Geometry(**s.kwargs())
    clean = og.forward(c)
    c = c * (4.0 / clean.max())
    clean = clean * (4.0 / clean.max())
    y = phantoms.poisson_log_sinogram(clean, 1e5, 33)
    return c.astype(np.float32), y


def large_inputs():
    s = workloads.LARGE
    y = phantoms.uniform((s.n_views, s.n_det), 77, 0.0, 4.0)
    rng = np.random.default_rng(78)
    pix = np.stack([rng.integers(0, s.n, 256), rng.integers(0, s.n, 256)], axis=1)
    return y, pix


def make_reduced():
    s = REDUCED
    _, y = reduced_inputs()
    og = oracle.Geometry(**s.kwargs())
    t = time.time()
    x = og.sirt(y.astype(np.float64), 50)
    print(f"reduced SIRT-50: {time.time() - t:.1f} s", flush=True)
    np.savez(os.path.join(HERE, "sirt50_reduced.npz"), x=x)


def make_large():
    s = workloads.LARGE
    y, pix = large_inputs()
    y = y.astype(np.float64)
    og = oracle.Geometry(**s.kwargs())
    t = time.time()
    row = og.forward(np.ones((s.n, s.n)))
    print(f"row sums {time.time() - t:.0f} s", flush=True)
    col = og.back(np.ones((s.n_views, s.n_det)))
    print(f"column sums {time.time() - t:.0f} s", flush=True)
    R = np.where(row != 0, 1.0 / np.where(row != 0, row, 1.0), 0.0)
    C = np.where(col != 0, 1.0 / np.where(col != 0, col, 1.0), 0.0)
    x1 = C * og.back(R * y)                      # step 1 from zero
    print(f"step 1 {time.time() - t:.0f} s", flush=True)
    r = R * (y - og.forward(x1))
    print(f"forward of x1 {time.time() - t:.0f} s", flush=True)
    vals = np.array([x1[j, i] + C[j, i] * og.back_pixel(r, i, j) for i, j in pix])
    np.savez(os.path.join(HERE, "sirt2_large_sampled.npz"), pix=pix, x2=vals,
             x1=np.array([x1[j, i] for i, j in pix]))
    print(f"large done {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--skip-reduced", action="store_true")
    a = ap.parse_args()
    oracle.build(force=False)
    if not a.skip_reduced:
        make_reduced()
    if not a.skip_large:
        make_large()
