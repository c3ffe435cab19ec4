"""GPU parity of the geometry variants against the FP64 oracle: the arc
detector, parallel beams and a cell pitch different from the cell width.

Same bar as the flat-detector parity tests: relative L2 error <= 1e-5 for
forward and back projection on identical FP32-rounded inputs, dense oracle
on small scans (every (ray, pixel) pair), ragged tiles and odd cell counts,
adjoint identity through the FP64 kernels, SIRT against the oracle's SIRT,
the non-zero count, and grouped SIRT steps over jobs of mixed beams.
"""
import math

import numpy as np
import pytest

from paper_1907_10526_amd import phantoms, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
MODES = {"flat": 0, "parallel": 1, "arc": 2}   # oracle modes


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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


def _pair(oracle_mod, fp, beam, pitch=None, **kw):
    og = oracle_mod.Geometry(**kw, det_spacing=pitch, mode=MODES[beam])
    gg = fp.Geometry(**kw, beam=beam, det_pitch=pitch)
    return og, gg


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check_pair(torch, og, gg, seed, label):
    img = phantoms.uniform((gg.ny, gg.nx), seed, 0.0, 1.0)
    y = gg.forward(_gpu(torch, img)).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    ef = rel_l2(y, y_ref)
    sino = phantoms.uniform((gg.n_views, gg.n_det), seed + 1, 0.0, 1.0)
    z = gg.back(_gpu(torch, sino)).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    eb = rel_l2(z, z_ref)
    print(f"{label}: forward rel-L2 {ef:.3e}, back rel-L2 {eb:.3e}", flush=True)
    assert np.linalg.norm(y_ref) > 0 and np.linalg.norm(z_ref) > 0
    assert ef <= TOL and eb <= TOL, (ef, eb)


@pytest.mark.parametrize("beam", ["arc", "parallel"])
def test_small_scan(oracle_mod, fp, torch_cuda, beam):
    s = workloads.SMALL
    og, gg = _pair(oracle_mod, fp, beam, **s.kwargs())
    _check_pair(torch_cuda, og, gg, 21, f"{beam} small scan")


@pytest.mark.parametrize("beam", ["arc", "parallel", "flat"])
@pytest.mark.parametrize("nx,ny,nd,pitch,width,dsc,dsd,pixel", [
    (37, 23, 77, 0.8, 0.9, 60.0, 130.0, 1.0),     # ragged tiles, odd cells, overlapping cells
    (16, 48, 40, 1.9, 1.7, 80.0, 96.0, 1.0),      # tall image, gaps between cells
    (48, 48, 96, 0.41, 0.41, 30.0, 55.0, 0.37),   # pixel size not one, wide fan
    (1, 1, 9, 0.5, 0.5, 3.0, 6.0, 1.0),           # single pixel next to the source
])
def test_ragged_shapes(oracle_mod, fp, torch_cuda, beam, nx, ny, nd, pitch, width, dsc, dsd, pixel):
    rng = np.random.default_rng(nx * 1000 + ny)
    angs = np.concatenate([[0.0, math.pi / 2, math.pi, 1.5 * math.pi, math.pi / 4],
                           rng.uniform(0.0, 2 * math.pi, 28)])
    kw = dict(nx=nx, ny=ny, pixel=pixel, dsc=dsc, dsd=dsd, angles=angs, n_det=nd, det_width=width)
    og, gg = _pair(oracle_mod, fp, beam, pitch=pitch, **kw)
    _check_pair(torch_cuda, og, gg, nx + ny, f"{beam} {nx}x{ny} pitch {pitch} width {width}")


@pytest.mark.parametrize("beam", ["arc", "parallel"])
def test_f64_kernels_match_oracle_and_adjoint(oracle_mod, fp, torch_cuda, beam):
    """The FP64 instantiation agrees with the oracle to FP64 rounding, which
    pins the GPU's geometry for the variant exactly, and is adjoint to 1e-12."""
    torch = torch_cuda
    angs = phantoms.view_angles(24)
    kw = dict(nx=40, ny=33, pixel=0.9, dsc=70.0, dsd=150.0, angles=angs, n_det=70, det_width=1.1)
    og, gg = _pair(oracle_mod, fp, beam, pitch=1.05, **kw)
    c = phantoms.uniform((33, 40), 31).astype(np.float64)
    y = phantoms.uniform((24, 70), 32).astype(np.float64)
    fy = gg.forward(torch.from_numpy(c).cuda()).cpu().numpy()
    bz = gg.back(torch.from_numpy(y).cuda()).cpu().numpy()
    ef, eb = rel_l2(fy, og.forward(c)), rel_l2(bz, og.back(y))
    print(f"{beam} FP64 kernels vs oracle: forward {ef:.2e}, back {eb:.2e}", flush=True)
    assert ef < 1e-10 and eb < 1e-10
    lhs, rhs = float(np.sum(fy * y)), float(np.sum(c * bz))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("beam", ["arc", "parallel"])
def test_sirt_matches_oracle(oracle_mod, fp, torch_cuda, beam):
    torch = torch_cuda
    angs = phantoms.view_angles(60)
    kw = dict(nx=48, ny=48, pixel=1.0, dsc=100.0, dsd=200.0, angles=angs, n_det=100, det_width=1.2)
    og, gg = _pair(oracle_mod, fp, beam, **kw)
    x_true = phantoms.ellipses(48, 5, 7).astype(np.float32)
    y = og.forward(x_true.astype(np.float64)).astype(np.float32)
    x_ref = og.sirt(y.astype(np.float64), 20)
    x = torch.zeros((48, 48), device="cuda")
    yg = _gpu(torch, y)
    w = torch.empty_like(yg)
    for _ in range(20):
        gg.sirt_step(x, yg, 1.0, w)
    err = rel_l2(x.cpu().numpy(), x_ref)
    print(f"{beam} SIRT-20 rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("beam", ["arc", "parallel"])
def test_count_nonzero(oracle_mod, fp, torch_cuda, beam):
    """Non-zero entries counted by the GPU's own enumeration.  The views are
    turned off the axes: at an axis-aligned parallel view with pitch = width
    the support edge |s'| = hab + tau/2 falls exactly on pixel centres, where
    the spline is exactly zero and rounding alone decides whether an entry
    reads as zero."""
    kw = workloads.SMALL.kwargs()
    kw["angles"] = kw["angles"] + 0.0123
    og, gg = _pair(oracle_mod, fp, beam, **kw)
    a, b = gg.count_nonzero(), og.count_nonzero()
    assert abs(a - b) <= 1e-4 * b, (a, b)


def test_grouped_steps_with_mixed_beams(fp, torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(44)
    specs = []
    for k, beam in enumerate(["flat", "arc", "parallel", "arc", "flat", "parallel", "arc"]):
        n = int(rng.choice([24, 40, 64]))
        nv = int(rng.choice([30, 45]))
        specs.append((beam, dict(nx=n, ny=n, pixel=1.0, dsc=3.0 * n, dsd=4.5 * n,
                                 angles=2 * math.pi * np.arange(nv) / nv, n_det=2 * n + k,
                                 det_width=float(rng.choice([0.9, 1.2])),
                                 det_pitch=float(rng.choice([0.9, 1.0, 1.2])))))
    geoms = [fp.Geometry(**kw, beam=beam) for beam, kw in specs]
    ys = [_gpu(torch, phantoms.uniform((g.n_views, g.n_det), 300 + k, 0.0, 3.0))
          for k, g in enumerate(geoms)]
    xs = [torch.zeros((g.ny, g.nx), device="cuda") for g in geoms]
    ws = [torch.empty_like(y) for y in ys]
    for g in geoms:
        fp.fp_sirt_prepare(g.handle)
    for _ in range(3):
        fp.fp_sirt_step_multi([(g.handle, x, y, w, 0.8) for g, x, y, w in zip(geoms, xs, ys, ws)])
    torch.cuda.synchronize()
    for k, (g, y) in enumerate(zip(geoms, ys)):
        x = torch.zeros((g.ny, g.nx), device="cuda")
        w = torch.empty_like(y)
        for _ in range(3):
            g.sirt_step(x, y, 0.8, w)
        err = float((xs[k].double() - x.double()).norm() / x.double().norm())
        assert err <= 1e-5, (k, specs[k][0], err)
