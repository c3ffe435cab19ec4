"""The octant form of the back projection.

A quarter-turn symmetric scan that the reflection across the image diagonal
x = y also leaves unchanged (V a multiple of 8, view Q - v at pi/2 minus the
angle of view v, Q = V/4; e.g. V views uniform over 2 pi from angle 0) has
symmetry order 8: the back projection of one image evaluates each entry of
the base views 0 .. Q/2 once for its four quarter turns and their four
reflections (batches and the forward projection run in the quarter-turn
form).
Both are checked against the dense FP64 oracle (which evaluates every view
on its own) for all beams, on scans down to the smallest (Q = 2, where both
base views are their own reflections), against the plain form of the same
scan (views listed in reverse order), for batches, for SIRT, and for the
symmetry detection.
"""
import numpy as np
import pytest

from paper_1907_10526_amd import phantoms

pytestmark = pytest.mark.gpu

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


def _kw(n, nv, nd, width, offset=0.0):
    angs = 2.0 * np.pi * np.arange(nv) / nv + offset
    return dict(nx=n, ny=n, pixel=1.0, dsc=3.0 * n, dsd=4.5 * n, angles=angs, n_det=nd,
                det_width=width)


@pytest.mark.parametrize("beam", ["flat", "arc", "parallel"])
@pytest.mark.parametrize("n,nv,nd,width,pitch", [
    (64, 48, 130, 1.3, None),    # aligned image
    (37, 40, 77, 0.9, 0.8),      # ragged tiles, odd cells, overlapping cells, odd Q
    (50, 8, 61, 1.1, None),      # Q = 2: both base views are their own reflections
    (33, 16, 70, 0.7, 0.75),     # Q = 4: one reflected base view
    (1, 8, 9, 0.5, None),        # one pixel
])
def test_against_dense_oracle(oracle_mod, fp, torch_cuda, beam, n, nv, nd, width, pitch):
    torch = torch_cuda
    kw = _kw(n, nv, nd, width)
    og = oracle_mod.Geometry(**kw, det_spacing=pitch, mode=MODES[beam])
    gg = fp.Geometry(**kw, beam=beam, det_pitch=pitch)
    assert gg.symmetry() == 8
    img = phantoms.uniform((n, n), 171, 0.0, 1.0)
    y = gg.forward(torch.from_numpy(img).cuda()).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    sino = phantoms.uniform((nv, nd), 172, 0.0, 1.0)
    z = gg.back(torch.from_numpy(sino).cuda()).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    ef, eb = rel_l2(y, y_ref), rel_l2(z, z_ref)
    # every view row and every pixel, not only the norm
    row = np.abs(y - y_ref).max(axis=1) / np.abs(y_ref).max()
    print(f"octant {beam} {n}^2 x {nv} x {nd}: forward rel-L2 {ef:.3e}, back rel-L2 {eb:.3e}, "
          f"worst view max-abs {row.max():.2e}", flush=True)
    assert ef <= 1e-5 and eb <= 1e-5, (ef, eb)
    assert row.max() <= 1e-5
    assert np.abs(z - z_ref).max() <= 1e-5 * np.abs(z_ref).max()


@pytest.mark.parametrize("beam", ["flat", "arc", "parallel"])
def test_matches_plain_form(fp, torch_cuda, beam):
    """The same 160^2 x 360-view scan with its views listed in reverse (plain
    form) and in order (octant back projection image by image, quarter-turn
    form for the batch of three): view by view and pixel by pixel to FP32
    rounding; repeated calls are bitwise equal."""
    torch = torch_cuda
    n, nv, nd = 160, 360, 330
    kw = _kw(n, nv, nd, 1.0)
    go = fp.Geometry(**kw, beam=beam)
    gp = fp.Geometry(**dict(kw, angles=kw["angles"][::-1].copy()), beam=beam)
    assert go.symmetry() == 8 and gp.symmetry() == 1
    imgs = torch.from_numpy(np.stack([phantoms.ellipses(n, 8, 180 + b) for b in range(3)])).cuda()
    yo = go.forward(imgs)
    yp = gp.forward(imgs).flip(1)
    ef = float((yo.double() - yp.double()).norm() / yp.double().norm())
    fr = float(((yo.double() - yp.double()).abs().amax(dim=2) / yp.double().abs().max()).max())
    sino = torch.from_numpy(np.stack([phantoms.uniform((nv, nd), 190 + b, 0.0, 1.0)
                                      for b in range(3)])).cuda()
    zo = go.back(sino)
    zp = gp.back(sino.flip(1).contiguous())
    eb = float((zo.double() - zp.double()).norm() / zp.double().norm())
    worst = 0.0
    for b in range(3):
        z1 = go.back(sino[b].contiguous())          # the octant form
        e1 = float((z1.double() - zp[b].double()).norm() / zp[b].double().norm())
        p1 = float((z1.double() - zp[b].double()).abs().max() / zp[b].double().abs().max())
        worst = max(worst, e1, p1)
        assert torch.equal(go.back(sino[b].contiguous()), z1)
        assert torch.equal(go.forward(imgs[b].contiguous()), yo[b])
    print(f"{beam} vs plain: forward {ef:.2e} (worst view {fr:.2e}), batch back {eb:.2e}, "
          f"octant back {worst:.2e}", flush=True)
    assert ef <= 1e-6 and eb <= 1e-6 and fr <= 1e-6 and worst <= 1e-6
    assert torch.equal(go.forward(imgs), yo) and torch.equal(go.back(sino), zo)


@pytest.mark.parametrize("beam", ["flat", "arc"])
def test_sirt(oracle_mod, fp, torch_cuda, beam):
    """20 SIRT steps (quarter-turn forward, octant back) against the oracle's
    SIRT, and the adjoint identity of the two operators."""
    torch = torch_cuda
    n, nv, nd = 80, 96, 170
    kw = _kw(n, nv, nd, 1.1)
    og = oracle_mod.Geometry(**kw, mode=MODES[beam])
    gg = fp.Geometry(**kw, beam=beam)
    assert gg.symmetry() == 8
    c = torch.from_numpy(phantoms.uniform((n, n), 173)).cuda()
    yv = torch.from_numpy(phantoms.uniform((nv, nd), 174)).cuda()
    lhs = float((gg.forward(c).double() * yv.double()).sum())
    rhs = float((c.double() * gg.back(yv).double()).sum())
    # FP32 rounding of either side is bounded relative to the sum without
    # cancellation, sum_j (A |c|)_j |yv_j| (random signs leave <A c, y> at about
    # 1e-3 of it)
    scale = float((gg.forward(c.abs()).double() * yv.abs().double()).sum())
    assert abs(lhs - rhs) <= 1e-8 * scale, (lhs, rhs, scale)
    truth = np.clip(phantoms.ellipses(n, 6, 175), 0.0, None).astype(np.float64)
    y = og.forward(truth).astype(np.float32)
    x_ref = og.sirt(y.astype(np.float64), 20)
    x = torch.zeros((n, n), device="cuda")
    yg = torch.from_numpy(y).cuda()
    w = torch.empty_like(yg)
    for _ in range(20):
        gg.sirt_step(x, yg, 1.0, w)
    err = rel_l2(x.cpu().numpy(), x_ref)
    print(f"octant {beam} SIRT-20 rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


def test_form_selection(fp, torch_cuda):
    """Symmetry order: 8 for a quarter-turn symmetric scan that the diagonal
    reflection also leaves unchanged, 4 for one it does not, 1 otherwise."""
    def vpe(nv=48, offset=0.0, **over):
        kw = _kw(64, nv, 130, 1.3, offset)
        kw.update(over)
        return fp.Geometry(**kw).symmetry()
    assert vpe() == 8
    assert vpe(nv=720) == 8
    assert vpe(offset=np.pi) == 8                   # the same view set
    assert vpe(nv=36) == 4                          # V % 8 == 4
    assert vpe(offset=0.3) == 4                     # quarter turns, no reflection
    assert vpe(offset=np.pi / 4) == 4               # reflection across x = -y only
    assert vpe(nx=64, ny=63) == 1                   # not square
    ang = 2.0 * np.pi * np.arange(48) / 48
    bent = ang.copy()
    bent[30] += 1e-9
    assert vpe(angles=bent) == 1
