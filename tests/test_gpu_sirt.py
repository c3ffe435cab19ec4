"""SIRT through the C ABI against the FP64 oracle.

* 50 steps from zero on a 256 x 256 scan with the large scan's proportions
  and Poisson-noisy data: rel-L2 of the iterate <= 1e-4 against the stored
  oracle iterate (tests/golden/sirt50_reduced.npz, written by
  make_sirt_golden.py from the oracle only).
* Two steps on the full 2048 x 2048 x 1440 x 2048 scan: sampled pixels of the
  iterate against stored oracle values.
* 50 steps from zero on the full scan with its Poisson-noisy data (the
  stored float32 log sinogram both sides read): the iterate at 16384 seeded
  pixels, along the two central rows and the central column, and its norm,
  against the stored oracle iterate (tests/golden/sirt50_large_*.npz, written
  by make_sirt_golden.py --large50 from the oracle only), rel-L2 <= 1e-4.
* 50 steps on the full scan: the R-weighted data residual never grows (a
  property of SIRT with 0 < lambda < 2), checked at several steps.
"""
import os
import sys

import numpy as np
import pytest

from paper_1907_10526_amd import phantoms, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def fp(torch_cuda):
    from paper_1907_10526_amd import fanproj
    return fanproj


def test_sirt50_reduced_matches_oracle(fp, torch_cuda):
    import make_sirt_golden as mg
    torch = torch_cuda
    path = os.path.join(GOLDEN, "sirt50_reduced.npz")
    ref = np.load(path)["x"]
    s = mg.REDUCED
    _, y = mg.reduced_inputs()
    g = fp.Geometry(**s.kwargs())
    x = torch.zeros((s.n, s.n), dtype=torch.float32, device="cuda")
    yt = torch.from_numpy(y).cuda()
    work = torch.empty_like(yt)
    for _ in range(50):
        g.sirt_step(x, yt, 1.0, work)
    err = rel_l2(x.cpu().numpy(), ref)
    print(f"reduced SIRT-50 rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


def test_sirt2_large_sampled(fp, torch_cuda):
    import make_sirt_golden as mg
    torch = torch_cuda
    path = os.path.join(GOLDEN, "sirt2_large_sampled.npz")
    if not os.path.exists(path):
        pytest.skip("stored large-scan SIRT values not generated")
    ref = np.load(path)
    s = workloads.LARGE
    y, pix = mg.large_inputs()
    assert np.array_equal(pix, ref["pix"])
    g = fp.Geometry(**s.kwargs())
    x = torch.zeros((s.n, s.n), dtype=torch.float32, device="cuda")
    yt = torch.from_numpy(y).cuda()
    work = torch.empty_like(yt)
    g.sirt_step(x, yt, 1.0, work)
    x1 = x.cpu().numpy()
    g.sirt_step(x, yt, 1.0, work)
    x2 = x.cpu().numpy()
    got1 = np.array([x1[j, i] for i, j in pix])
    got2 = np.array([x2[j, i] for i, j in pix])
    e1, e2 = rel_l2(got1, ref["x1"]), rel_l2(got2, ref["x2"])
    print(f"large SIRT step 1 / 2 sampled rel-L2 {e1:.3e} / {e2:.3e}", flush=True)
    assert e1 <= 1e-5 and e2 <= 1e-5


def test_sirt50_large_matches_stored_oracle(fp, torch_cuda):
    import make_sirt_golden as mg
    torch = torch_cuda
    f_sino = os.path.join(GOLDEN, "sirt50_large_sino.npz")
    f_ref = os.path.join(GOLDEN, "sirt50_large_sampled.npz")
    if not (os.path.exists(f_sino) and os.path.exists(f_ref)):
        pytest.skip("stored 50-step large-scan SIRT iterate not generated")
    ref = np.load(f_ref)
    s = workloads.LARGE
    y = np.load(f_sino)["y"]
    assert y.dtype == np.float32 and y.shape == (s.n_views, s.n_det)
    pix = ref["pix"]
    assert np.array_equal(pix, mg.large50_sample_positions(s.n))
    g = fp.Geometry(**s.kwargs())
    x = torch.zeros((s.n, s.n), dtype=torch.float32, device="cuda")
    yt = torch.from_numpy(y).cuda()
    work = torch.empty_like(yt)
    for _ in range(int(ref["iters"])):
        g.sirt_step(x, yt, 1.0, work)
    xc = x.cpu().numpy().astype(np.float64)
    e_pix = rel_l2(xc[pix[:, 1], pix[:, 0]], ref["x"])
    e_rows = rel_l2(xc[ref["row_index"], :], ref["rows"])
    e_col = rel_l2(xc[:, int(ref["col_index"])], ref["col"])
    e_norm = abs(np.sqrt(np.sum(xc * xc)) / np.sqrt(float(ref["sumsq"])) - 1.0)
    print(f"large SIRT-{int(ref['iters'])} vs oracle: {len(pix)} pixels rel-L2 {e_pix:.3e}, "
          f"central rows {e_rows:.3e}, central column {e_col:.3e}, norm {e_norm:.3e} "
          f"(symmetry order {g.symmetry()})", flush=True)
    assert max(e_pix, e_rows, e_col, e_norm) <= 1e-4


def test_sirt50_large_residual_decreases(fp, torch_cuda):
    torch = torch_cuda
    s = workloads.LARGE
    g = fp.Geometry(**s.kwargs())
    scale = s.n / 64.0
    c = np.clip(phantoms.ellipses(s.n, 20, 3, (4.0 * scale, 20.0 * scale)), 0.0, None)
    ct = torch.from_numpy(c).cuda()
    clean = g.forward(ct)
    k = 4.0 / float(clean.max())
    clean = clean * k
    y = torch.from_numpy(phantoms.poisson_log_sinogram(clean.cpu().numpy(), 1e5, 33)).cuda()
    ones = torch.ones((s.n, s.n), device="cuda")
    row = g.forward(ones)
    R = torch.where(row != 0, 1.0 / torch.where(row != 0, row, torch.ones_like(row)), torch.zeros_like(row))
    x = torch.zeros((s.n, s.n), dtype=torch.float32, device="cuda")
    work = torch.empty_like(y)
    prev = float("inf")
    first = None
    for it in range(1, 51):
        g.sirt_step(x, y, 1.0, work)
        if it in (1, 2, 5, 10, 20, 50):
            r = y - g.forward(x)
            wres = float((R.double() * r.double() ** 2).sum())
            first = wres if first is None else first
            print(f"large SIRT step {it}: weighted residual {wres:.6e}", flush=True)
            assert wres <= prev * (1 + 1e-6)
            prev = wres
    assert prev < 0.5 * first
    # the iterate approaches the (scaled) phantom in the field of view
    xc = x.cpu().numpy()
    assert np.isfinite(xc).all()
