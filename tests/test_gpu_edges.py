"""Edge cases of the C ABI on the GPU: degenerate sizes, odd batch sizes,
unusual angles, rejected arguments and geometries beyond the on-chip
staging, each against the FP64 oracle or the documented error."""
import math

import numpy as np
import pytest

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


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("nv,nd", [(1, 1), (1, 64), (7, 1), (3, 2)])
def test_single_view_or_cell(oracle_mod, fp, torch_cuda, nv, nd):
    torch = torch_cuda
    angs = np.array([0.37, 1.9, 2.5, 3.3, 4.0, 5.1, 6.0])[:nv]
    kw = dict(nx=24, ny=24, pixel=1.0, dsc=60.0, dsd=120.0, angles=angs, n_det=nd, det_width=1.3)
    og, gg = oracle_mod.Geometry(**kw), fp.Geometry(**kw)
    img = phantoms.uniform((24, 24), 5, 0.0, 1.0)
    y = gg.forward(_gpu(torch, img)).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    assert rel_l2(y, y_ref) <= TOL
    sino = phantoms.uniform((nv, nd), 6, 0.0, 1.0)
    z = gg.back(_gpu(torch, sino)).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    assert rel_l2(z, z_ref) <= TOL


def test_unusual_angles(oracle_mod, fp, torch_cuda):
    """Negative, repeated and multi-turn angles, and exact axis angles."""
    torch = torch_cuda
    angs = np.array([-math.pi, -0.5, 0.0, 0.0, math.pi / 2, 7 * math.pi, 13.25, 2 * math.pi])
    kw = dict(nx=40, ny=31, pixel=0.8, dsc=70.0, dsd=110.0, angles=angs, n_det=90, det_width=0.9)
    og, gg = oracle_mod.Geometry(**kw), fp.Geometry(**kw)
    img = phantoms.uniform((31, 40), 7, 0.0, 1.0)
    y = gg.forward(_gpu(torch, img)).cpu().numpy()
    assert rel_l2(y, og.forward(img.astype(np.float64), dense=True)) <= TOL
    assert np.array_equal(y[2], y[3])            # repeated angle, same rays
    sino = phantoms.uniform((len(angs), 90), 8, 0.0, 1.0)
    z = gg.back(_gpu(torch, sino)).cpu().numpy()
    assert rel_l2(z, og.back(sino.astype(np.float64), dense=True)) <= TOL


def test_batch_thirteen_equals_single_images(fp, torch_cuda):
    """13 images run as chunks of 8, 4 and 1 images; every image's result is
    bitwise the one it gets alone, forward and back, FP32 and FP64."""
    torch = torch_cuda
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    imgs = _gpu(torch, np.stack([workloads.phantom(s, seed=300 + k) for k in range(13)]))
    y = gg.forward(imgs)
    z = gg.back(y)
    for k in range(13):
        assert torch.equal(gg.forward(imgs[k].contiguous()), y[k])
        assert torch.equal(gg.back(y[k].contiguous()), z[k])
    y64 = gg.forward(imgs.double())
    for k in (0, 8, 12):
        assert torch.equal(gg.forward(imgs[k].double().contiguous()), y64[k])


def test_zero_image_and_zero_sinogram(fp, torch_cuda):
    torch = torch_cuda
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    assert float(gg.forward(torch.zeros((s.n, s.n), device="cuda")).abs().max()) == 0.0
    assert float(gg.back(torch.zeros((s.n_views, s.n_det), device="cuda")).abs().max()) == 0.0


def test_cells_too_narrow_for_the_staging_are_rejected(fp, torch_cuda):
    """A geometry whose back-projection tiles span more cells than the LDS
    staging holds is refused at creation with FP_ERR_UNSUPPORTED."""
    angs = phantoms.view_angles(8)
    with pytest.raises(fp.FanprojError) as e:
        fp.Geometry(64, 64, 1.0, 128.0, 256.0, angs, 20000, 0.01)
    assert e.value.status == fp.FP_ERR_UNSUPPORTED
    assert "on-chip staging" in str(e.value)
    # the device is still usable
    g = fp.Geometry(8, 8, 1.0, 20.0, 40.0, angs, 16, 1.0)
    assert float(g.forward(torch_cuda.ones((8, 8), device="cuda")).sum()) > 0


def test_rejected_arguments(fp, torch_cuda):
    torch = torch_cuda
    import ctypes
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    img = torch.zeros((s.n, s.n), device="cuda")
    out = torch.empty((s.n_views, s.n_det), device="cuda")
    st = fp._lib.fp_forward(gg.handle, ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                            0, None)
    assert st == fp.FP_ERR_INVALID_ARG                       # batch 0
    with pytest.raises(ValueError):
        gg.forward(img.t())                                  # not contiguous
    with pytest.raises(ValueError):
        gg.forward(img.half())                               # wrong dtype
    with pytest.raises(ValueError):
        gg.back(torch.zeros((s.n_views, s.n_det + 1), device="cuda"))   # wrong shape
    with pytest.raises(fp.FanprojError):
        fp.fp_forward_reference(gg.handle, img.double(), out.double(), 1, quad_points=99)


def test_device_bytes_cover_the_sirt_weights(fp, torch_cuda):
    s = workloads.SMALL
    gg = fp.Geometry(**s.kwargs())
    before = gg.device_bytes()
    fp.fp_sirt_prepare(gg.handle)
    after = gg.device_bytes()
    assert before > 7 * 4 * s.n_views * s.n_det
    assert after >= before + 4 * (s.n_views * s.n_det + s.n * s.n)
