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
* ``sirt50_large_sino.npz`` and ``sirt50_large_sampled.npz``: the full-size
  SIRT workload itself.  The phantom is the 20-ellipse phantom of the large
  scan (seed 3, semi-axes 128-640 px) clipped at zero and scaled so that its
  largest line integral is 4; the data are Poisson counts (I0 = 1e5, seed 33)
  of its oracle sinogram, stored as the float32 log sinogram both sides read.
  The stored result is the oracle's 50th SIRT iterate from zero at 16384
  seeded pixels (seed 79), along the two central rows and the central column,
  plus its full-image sum of squares.  This is 103 full-size projections
  (about 3 hours on 8 threads with the cached-frame operators); the run
  checkpoints every iteration into ``--checkpoint-dir`` and resumes from it.
"""
from __future__ import annotations

import argparse
import os
import sys
import tempfile
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


def sirt_weights(og, cached=True):
    """R = 1 / (A 1) and C = 1 / (A^T 1), with 1/0 read as 0 (the oracle's
    SIRT weights, computed with its operators)."""
    row = og.forward(np.ones((og.ny, og.nx)), cached=cached)
    col = og.back(np.ones((og.n_views, og.n_det)), cached=cached)
    R = np.where(row != 0.0, 1.0 / np.where(row != 0.0, row, 1.0), 0.0)
    C = np.where(col != 0.0, 1.0 / np.where(col != 0.0, col, 1.0), 0.0)
    return R, C


def sirt_step(og, x, y, R, C, relaxation=1.0, cached=True):
    """One SIRT step x + lambda C (A^T (R (y - A x))), elementwise in the
    order of the oracle's own SIRT loop, so the two agree bitwise."""
    r = R * (y - og.forward(x, cached=cached))
    z = og.back(r, cached=cached)
    return x + relaxation * C * z


LARGE50_ITERS = 50
LARGE50_PIXELS = 16384


def large50_sample_positions(n):
    """16384 seeded pixel positions (column, row) of the stored iterate."""
    rng = np.random.default_rng(79)
    return np.stack([rng.integers(0, n, LARGE50_PIXELS), rng.integers(0, n, LARGE50_PIXELS)], axis=1)


def make_large50(ckpt):
    s = workloads.LARGE
    og = oracle.Geometry(**s.kwargs())
    os.makedirs(ckpt, exist_ok=True)
    t = time.time()
    f_sino = os.path.join(HERE, "sirt50_large_sino.npz")
    if os.path.exists(f_sino):
        y = np.load(f_sino)["y"]
    else:
        c = np.clip(workloads.phantom(s).astype(np.float64), 0.0, None)
        clean = og.forward(c, cached=True)
        scale = 4.0 / clean.max()
        y = phantoms.poisson_log_sinogram(clean * scale, 1e5, 33)
        np.savez_compressed(f_sino, y=y, scale=np.float64(scale))
        print(f"clean sinogram and noise {time.time() - t:.0f} s", flush=True)
    y64 = y.astype(np.float64)
    f_w = os.path.join(ckpt, "weights.npz")
    if os.path.exists(f_w):
        w = np.load(f_w)
        R, C = w["R"], w["C"]
    else:
        R, C = sirt_weights(og)
        np.savez(f_w, R=R, C=C)
        print(f"weights {time.time() - t:.0f} s", flush=True)
    x, it0 = np.zeros((s.n, s.n)), 0
    for it in range(LARGE50_ITERS, 0, -1):
        f = os.path.join(ckpt, f"x{it:02d}.npy")
        if os.path.exists(f):
            x, it0 = np.load(f), it
            break
    for it in range(it0 + 1, LARGE50_ITERS + 1):
        x = sirt_step(og, x, y64, R, C)
        np.save(os.path.join(ckpt, f"x{it:02d}.npy.tmp.npy"), x)
        os.replace(os.path.join(ckpt, f"x{it:02d}.npy.tmp.npy"), os.path.join(ckpt, f"x{it:02d}.npy"))
        if it > 1 and os.path.exists(os.path.join(ckpt, f"x{it - 1:02d}.npy")):
            os.remove(os.path.join(ckpt, f"x{it - 1:02d}.npy"))
        print(f"iteration {it} {time.time() - t:.0f} s", flush=True)
    pix = large50_sample_positions(s.n)
    mid = s.n // 2
    np.savez(os.path.join(HERE, "sirt50_large_sampled.npz"),
             iters=np.int32(LARGE50_ITERS), pix=pix, x=x[pix[:, 1], pix[:, 0]],
             rows=x[[mid - 1, mid], :], row_index=np.array([mid - 1, mid]),
             col=x[:, mid], col_index=np.int32(mid), sumsq=np.float64(np.sum(x * x)))
    print(f"large 50-step SIRT done {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--skip-reduced", action="store_true")
    ap.add_argument("--large50", action="store_true",
                    help="only the 50-step full-size SIRT iterate (hours of CPU)")
    ap.add_argument("--checkpoint-dir", default=os.path.join(tempfile.gettempdir(), "sirt50_large_ckpt"))
    a = ap.parse_args()
    oracle.build(force=False)
    if a.large50:
        make_large50(a.checkpoint_dir)
        sys.exit(0)
    if not a.skip_reduced:
        make_reduced()
    if not a.skip_large:
        make_large()
