"""GPU parity: the HIP projector through the C ABI against the FP64 oracle.

Both sides get the same FP32-rounded inputs; the tolerance is the relative
L2 error 1e-5 for forward and back projection (1e-4 after 50 SIRT steps).
Small scans are compared in full (dense oracle where cheap), the full-size
scans on sampled outputs that the oracle computes one at a time.
"""
import math

import numpy as np
import pytest

import exact_geometry as eg
from paper_1907_10526_amd import phantoms, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def _pair(oracle_mod, fp, **kw):
    og = oracle_mod.Geometry(**kw)
    gg = fp.Geometry(**kw)
    return og, gg


def _to_gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_small_scan_forward_and_back(oracle_mod, fp, torch_cuda):
    torch = torch_cuda
    s = workloads.SMALL
    og, gg = _pair(oracle_mod, fp, **s.kwargs())
    img = workloads.phantom(s)
    y = gg.forward(_to_gpu(torch, img)).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    err = rel_l2(y, y_ref)
    print(f"small forward rel-L2 {err:.3e} max {np.abs(y - y_ref).max():.3e}", flush=True)
    assert err <= TOL
    sino = phantoms.uniform((s.n_views, s.n_det), 12)
    z = gg.back(_to_gpu(torch, sino)).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    err = rel_l2(z, z_ref)
    print(f"small back rel-L2 {err:.3e} max {np.abs(z - z_ref).max():.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("nx,ny,nd,width,dsc,dsd", [
    (37, 23, 77, 0.9, 60.0, 130.0),     # ragged tiles, odd cell count
    (16, 48, 40, 1.7, 80.0, 96.0),      # tall image, wide cells, low magnification
    (1, 1, 9, 0.5, 3.0, 6.0),           # the paper's single-pixel set-up (Sec. V-A)
])
def test_ragged_shapes_against_dense_oracle(oracle_mod, fp, torch_cuda, nx, ny, nd, width, dsc, dsd):
    torch = torch_cuda
    rng = np.random.default_rng(nx * 1000 + ny)
    angs = np.concatenate([[0.0, math.pi / 2, math.pi, 1.5 * math.pi, math.pi / 4],
                           rng.uniform(0.0, 2 * math.pi, 28)])
    kw = dict(nx=nx, ny=ny, pixel=1.0, dsc=dsc, dsd=dsd, angles=angs, n_det=nd, det_width=width)
    og, gg = _pair(oracle_mod, fp, **kw)
    img = phantoms.uniform((ny, nx), 3, 0.0, 1.0)
    y = gg.forward(_to_gpu(torch, img)).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    assert rel_l2(y, y_ref) <= TOL, rel_l2(y, y_ref)
    sino = phantoms.uniform((len(angs), nd), 4, 0.0, 1.0)
    z = gg.back(_to_gpu(torch, sino)).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    assert rel_l2(z, z_ref) <= TOL, rel_l2(z, z_ref)


def test_pixel_size_not_one(oracle_mod, fp, torch_cuda):
    torch = torch_cuda
    angs = phantoms.view_angles(40)
    kw = dict(nx=48, ny=48, pixel=0.37, dsc=30.0, dsd=55.0, angles=angs, n_det=96, det_width=0.41)
    og, gg = _pair(oracle_mod, fp, **kw)
    img = phantoms.uniform((48, 48), 5, 0.0, 1.0)
    y = gg.forward(_to_gpu(torch, img)).cpu().numpy()
    assert rel_l2(y, og.forward(img.astype(np.float64))) <= TOL
    sino = phantoms.uniform((40, 96), 6, 0.0, 1.0)
    z = gg.back(_to_gpu(torch, sino)).cpu().numpy()
    assert rel_l2(z, og.back(sino.astype(np.float64))) <= TOL


def test_adjoint_identity_gpu(fp, torch_cuda):
    torch = torch_cuda
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    c = _to_gpu(torch, phantoms.uniform((s.n, s.n), 11))
    y = _to_gpu(torch, phantoms.uniform((s.n_views, s.n_det), 12))
    lhs = float((gg.forward(c).double() * y.double()).sum())
    rhs = float((c.double() * gg.back(y).double()).sum())
    # FP32 rounding of either side is bounded relative to the sum without
    # cancellation, sum_j (A |c|)_j |y_j| (random signs leave <A c, y> at about
    # 1e-3 of it)
    scale = float((gg.forward(c.abs()).double() * y.abs().double()).sum())
    assert abs(lhs - rhs) <= 1e-8 * scale, (lhs, rhs, scale)


def test_deterministic_and_batch_consistent(fp, torch_cuda):
    torch = torch_cuda
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    imgs = np.stack([workloads.phantom(s, seed=100 + k) for k in range(7)])
    x = _to_gpu(torch, imgs)
    yb = gg.forward(x)
    ya = gg.forward(x)
    assert torch.equal(ya, yb)
    for k in range(7):
        assert torch.equal(gg.forward(x[k].contiguous()), yb[k])
    sinos = _to_gpu(torch, np.stack([phantoms.uniform((s.n_views, s.n_det), 200 + k) for k in range(7)]))
    zb = gg.back(sinos)
    assert torch.equal(zb, gg.back(sinos))
    for k in range(7):
        assert torch.equal(gg.back(sinos[k].contiguous()), zb[k])


def _sample(rng, count, hi0, hi1):
    return [(int(rng.integers(0, hi0)), int(rng.integers(0, hi1))) for _ in range(count)]


@pytest.mark.parametrize("name,nray,npix", [("medium", 40, 40), ("large", 12, 24)])
def test_full_size_sampled(oracle_mod, fp, torch_cuda, name, nray, npix):
    torch = torch_cuda
    s = workloads.SCANS[name]
    og, gg = _pair(oracle_mod, fp, **s.kwargs())
    img = workloads.phantom(s)
    y = gg.forward(_to_gpu(torch, img)).cpu().numpy()
    rng = np.random.default_rng(9)
    img64 = img.astype(np.float64)
    rays = _sample(rng, nray, s.n_views, s.n_det)
    # rays near the centre of the detector cross the whole image
    rays += [(v, s.n_det // 2 + int(rng.integers(-20, 20))) for v, _ in _sample(rng, nray // 2, s.n_views, 1)]
    got = np.array([y[v, m] for v, m in rays])
    ref = np.array([og.forward_ray(img64, v, m) for v, m in rays])
    err = rel_l2(got, ref)
    print(f"{name} forward sampled rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
    sino = phantoms.uniform((s.n_views, s.n_det), 13, 0.0, 1.0)
    z = gg.back(_to_gpu(torch, sino)).cpu().numpy()
    sino64 = sino.astype(np.float64)
    pix = _sample(rng, npix, s.n, s.n) + [(0, 0), (s.n - 1, s.n - 1), (s.n // 2, s.n // 2)]
    got = np.array([z[j, i] for i, j in pix])
    ref = np.array([og.back_pixel(sino64, i, j) for i, j in pix])
    err = rel_l2(got, ref)
    print(f"{name} back sampled rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("beam", ["flat", "arc", "parallel"])
def test_ragged_single_group_sampled(oracle_mod, fp, torch_cuda, beam):
    """1040 x 1030 pixels: 65 x 33 = 2145 back-projection tiles, so one view
    group and a tile count that is not a multiple of the XCD count (the
    work-group order then gives the XCDs bands of 269 and 268 tiles); ragged
    tiles on two edges.  Sampled against the oracle, corners and tile edges
    included."""
    torch = torch_cuda
    nx, ny, nv = 1040, 1030, 30
    nd = 1500 if beam == "parallel" else 2200
    angles = 2.0 * np.pi * np.arange(nv) / nv + 0.1
    kw = dict(nx=nx, ny=ny, pixel=1.0, dsc=1600.0, dsd=2400.0, angles=angles, n_det=nd,
              det_width=1.0)
    mode = {"flat": 0, "parallel": 1, "arc": 2}[beam]   # oracle modes
    og = oracle_mod.Geometry(**kw, mode=mode)
    gg = fp.Geometry(**kw, beam=beam)   # 8 work-groups per CU fill the chip: one group
    img = phantoms.uniform((ny, nx), 21, 0.0, 1.0)
    y = gg.forward(_to_gpu(torch, img)).cpu().numpy()
    rng = np.random.default_rng(31)
    rays = _sample(rng, 16, nv, nd) + [(v, nd // 2 + int(rng.integers(-30, 30))) for v in (0, 7, 19)]
    got = np.array([y[v, m] for v, m in rays])
    ref = np.array([og.forward_ray(img.astype(np.float64), v, m) for v, m in rays])
    err = rel_l2(got, ref)
    print(f"{beam} ragged single-group forward sampled rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
    sino = phantoms.uniform((nv, nd), 22, 0.0, 1.0)
    z = gg.back(_to_gpu(torch, sino)).cpu().numpy()
    pix = _sample(rng, 30, nx, ny) + [(0, 0), (nx - 1, ny - 1), (nx - 1, 0), (0, ny - 1),
                                       (15, 31), (16, 32), (1039, 1023), (1024, 1024)]
    got = np.array([z[j, i] for i, j in pix])
    ref = np.array([og.back_pixel(sino.astype(np.float64), i, j) for i, j in pix])
    err = rel_l2(got, ref)
    print(f"{beam} ragged single-group back sampled rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_medium_disk_closed_form(fp, torch_cuda):
    """A uniform disk of radius 200 px projects to the bin average of
    2 sqrt(r^2 - d^2); the GPU result is within the pixelisation error."""
    torch = torch_cuda
    s = workloads.MEDIUM
    gg = fp.Geometry(**s.kwargs())
    y = gg.forward(_to_gpu(torch, workloads.disk_phantom(s))).cpu().numpy()
    views = [0, 90, 137, 400]
    ref = np.array([[eg.disk_fan_projection(s.view_angles()[v], s.dsc, s.dsd,
                                            (m - 0.5 * (s.n_det - 1)) * s.det_width, s.det_width, 200.0)
                     for m in range(s.n_det)] for v in views])
    err = rel_l2(y[views], ref)
    print(f"medium disk rel-L2 vs closed form {err:.3e}", flush=True)
    assert err < 2e-3


def test_sirt_small_matches_oracle(oracle_mod, fp, torch_cuda):
    torch = torch_cuda
    s = workloads.SMALL
    og, gg = _pair(oracle_mod, fp, **s.kwargs())
    truth = np.clip(workloads.phantom(s), 0.0, None).astype(np.float64) * 0.05
    clean = og.forward(truth)
    y = phantoms.poisson_log_sinogram(clean, 1e5, 33)
    x = torch.zeros((s.n, s.n), dtype=torch.float32, device="cuda")
    yt = _to_gpu(torch, y)
    work = torch.empty_like(yt)
    for _ in range(50):
        gg.sirt_step(x, yt, 1.0, work)
    x_ref = og.sirt(y.astype(np.float64), 50)
    err = rel_l2(x.cpu().numpy(), x_ref)
    print(f"small SIRT-50 rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


def test_count_nonzero_matches_oracle(oracle_mod, fp, torch_cuda):
    s = workloads.SMALL
    og, gg = _pair(oracle_mod, fp, **s.kwargs())
    got, ref = gg.count_nonzero(), og.count_nonzero()
    assert abs(got - ref) <= 1e-4 * ref, (got, ref)


def test_rejects_host_pointer(fp, torch_cuda):
    torch = torch_cuda
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    host = np.zeros((s.n, s.n), dtype=np.float32)
    out = torch.empty((s.n_views, s.n_det), device="cuda")
    import ctypes
    st = fp._lib.fp_forward(gg.handle, ctypes.c_void_p(host.ctypes.data), ctypes.c_void_p(out.data_ptr()),
                            1, None)
    assert st == fp.FP_ERR_INVALID_ARG
    assert "device memory" in fp.fp_last_error()
    # the geometry still works afterwards
    y = gg.forward(torch.zeros((s.n, s.n), device="cuda"))
    assert float(y.abs().max()) == 0.0


def test_medium_full_elementwise(oracle_mod, fp, torch_cuda):
    """The 512 x 512, 720-view, 1024-cell pair compared element by element
    with the oracle's full forward and back projections (every ray and
    every pixel): relative L2 <= 1e-5 and the largest deviation <= 1e-5 of
    the largest value; the GPU's non-zero count (the unit the throughput is
    priced in) equals the oracle's to 1e-4."""
    torch = torch_cuda
    s = workloads.MEDIUM
    og, gg = _pair(oracle_mod, fp, **s.kwargs())
    img = workloads.phantom(s)
    y = gg.forward(_to_gpu(torch, img)).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), cached=True)
    ef, mf = rel_l2(y, y_ref), float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
    sino = phantoms.uniform((s.n_views, s.n_det), 13, 0.0, 1.0)
    z = gg.back(_to_gpu(torch, sino)).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), cached=True)
    eb, mb = rel_l2(z, z_ref), float(np.abs(z - z_ref).max() / np.abs(z_ref).max())
    print(f"medium full: forward rel-L2 {ef:.3e} (max {mf:.3e} of peak), "
          f"back rel-L2 {eb:.3e} (max {mb:.3e} of peak)", flush=True)
    assert ef <= TOL and mf <= TOL
    assert eb <= TOL and mb <= TOL
    got, ref = gg.count_nonzero(), og.count_nonzero()
    print(f"medium non-zero entries: GPU {got}, oracle {ref}", flush=True)
    assert abs(got - ref) <= 1e-4 * ref, (got, ref)
