"""The quarter-turn form of the projections.

A square image scanned with views in quadruples a quarter turn apart (view
v + k V/4 at the angle of view v plus k pi/2, e.g. V views uniform over
2 pi with V a multiple of 4) takes the quarter-turn form: each entry is
evaluated once for four views, on the image turned by k quarter turns.  It
is checked here against the dense FP64 oracle (which evaluates every view on
its own), against the plain form of the same scan (the views listed in
reverse order, which the library does not recognise as quarter turns), for
batches split over launches, SIRT, the adjoint identity and determinism.
The scans here start at angles that the diagonal reflection does not map
onto the view set (or have V % 8 == 4), so they take the quarter-turn form
and not the octant form.
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


def _kw(n, nv, nd, width, pitch=None, offset=0.0, pixel=1.0):
    angs = 2.0 * np.pi * np.arange(nv) / nv + offset
    return dict(nx=n, ny=n, pixel=pixel, dsc=3.0 * n * pixel, dsd=4.5 * n * pixel, angles=angs,
                n_det=nd, det_width=width), pitch


@pytest.mark.parametrize("beam", ["flat", "arc", "parallel"])
@pytest.mark.parametrize("n,nv,nd,width,pitch,offset", [
    (64, 48, 130, 1.3, None, 0.05),     # aligned image
    (37, 36, 77, 0.9, 0.8, 0.3),        # ragged tiles, odd cells, overlapping cells, offset views
    (1, 8, 9, 0.5, None, 0.1),          # one pixel
])
def test_against_dense_oracle(oracle_mod, fp, torch_cuda, beam, n, nv, nd, width, pitch, offset):
    torch = torch_cuda
    kw, pitch = _kw(n, nv, nd, width, pitch, offset)
    og = oracle_mod.Geometry(**kw, det_spacing=pitch, mode=MODES[beam])
    gg = fp.Geometry(**kw, beam=beam, det_pitch=pitch)
    assert gg.symmetry() == 4
    img = phantoms.uniform((n, n), 71, 0.0, 1.0)
    y = gg.forward(torch.from_numpy(img).cuda()).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    sino = phantoms.uniform((nv, nd), 72, 0.0, 1.0)
    z = gg.back(torch.from_numpy(sino).cuda()).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    ef, eb = rel_l2(y, y_ref), rel_l2(z, z_ref)
    print(f"quarter {beam} {n}^2 x {nv} x {nd}: forward rel-L2 {ef:.3e}, back rel-L2 {eb:.3e}",
          flush=True)
    assert ef <= 1e-5 and eb <= 1e-5, (ef, eb)


@pytest.mark.parametrize("beam", ["flat", "arc", "parallel"])
def test_matches_plain_form(fp, torch_cuda, beam):
    """The same 160^2 x 360-view scan with its views listed in reverse (plain
    form) and in order (quarter-turn form): the results agree to FP32
    rounding, view by view and pixel by pixel, for a batch of three images
    (launch chunks of two and one)."""
    torch = torch_cuda
    n, nv, nd = 160, 360, 330
    kw, _ = _kw(n, nv, nd, 1.0, offset=np.pi / nv)   # half a view step
    gq = fp.Geometry(**kw, beam=beam)
    kw_rev = dict(kw, angles=kw["angles"][::-1].copy())
    gp = fp.Geometry(**kw_rev, beam=beam)
    assert gq.quarter_turn() and not gp.quarter_turn()
    assert gq.symmetry() == 4
    imgs = torch.from_numpy(np.stack([phantoms.ellipses(n, 8, 80 + b) for b in range(3)])).cuda()
    yq = gq.forward(imgs)
    yp = gp.forward(imgs).flip(1)
    ef = float((yq.double() - yp.double()).norm() / yp.double().norm())
    sino = torch.from_numpy(np.stack([phantoms.uniform((nv, nd), 90 + b, 0.0, 1.0)
                                      for b in range(3)])).cuda()
    zq = gq.back(sino)
    zp = gp.back(sino.flip(1).contiguous())
    eb = float((zq.double() - zp.double()).norm() / zp.double().norm())
    print(f"{beam} quarter vs plain: forward {ef:.2e}, back {eb:.2e}", flush=True)
    assert ef <= 1e-6 and eb <= 1e-6
    for b in range(3):
        assert torch.equal(gq.forward(imgs[b].contiguous()), yq[b])
        assert torch.equal(gq.back(sino[b].contiguous()), zq[b])
    assert torch.equal(gq.forward(imgs), yq) and torch.equal(gq.back(sino), zq)


def test_adjoint_and_sirt(oracle_mod, fp, torch_cuda):
    torch = torch_cuda
    kw, _ = _kw(96, 120, 200, 1.1, offset=0.2)
    og = oracle_mod.Geometry(**kw)
    gg = fp.Geometry(**kw)
    assert gg.symmetry() == 4
    c = torch.from_numpy(phantoms.uniform((96, 96), 73)).cuda()
    yv = torch.from_numpy(phantoms.uniform((120, 200), 74)).cuda()
    lhs = float((gg.forward(c).double() * yv.double()).sum())
    rhs = float((c.double() * gg.back(yv).double()).sum())
    # FP32 rounding of either side is bounded relative to the sum without
    # cancellation, sum_j (A |c|)_j |yv_j| (random signs leave <A c, y> at about
    # 1e-3 of it)
    scale = float((gg.forward(c.abs()).double() * yv.abs().double()).sum())
    assert abs(lhs - rhs) <= 1e-8 * scale, (lhs, rhs, scale)
    truth = np.clip(phantoms.ellipses(96, 6, 75), 0.0, None).astype(np.float64)
    y = og.forward(truth).astype(np.float32)
    x_ref = og.sirt(y.astype(np.float64), 20)
    x = torch.zeros((96, 96), device="cuda")
    yg = torch.from_numpy(y).cuda()
    w = torch.empty_like(yg)
    for _ in range(20):
        gg.sirt_step(x, yg, 1.0, w)
    err = rel_l2(x.cpu().numpy(), x_ref)
    print(f"quarter SIRT-20 rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


def test_form_selection(fp, torch_cuda):
    """The quarter-turn form is taken only for a square image whose views
    come in quarter-turn quadruples."""
    def q(**over):
        kw, _ = _kw(64, 48, 130, 1.3)
        kw.update(over)
        return fp.Geometry(**kw).quarter_turn()
    ang = 2.0 * np.pi * np.arange(48) / 48
    assert q()
    assert not q(nx=64, ny=63)                                  # not square
    assert not q(angles=2.0 * np.pi * np.arange(46) / 46)      # 46 views
    assert not q(angles=np.pi * np.arange(48) / 48)            # 48 views over pi
    bent = ang.copy()
    bent[30] += 1e-9
    assert not q(angles=bent)                                   # one view off
    assert q(angles=ang + 5.0)                                  # any first angle
    # quadruples listed view by view: v, v + 12, v + 24, v + 36 as
    # consecutive entries are quarter turns only in the blocked order
    assert not q(angles=ang.reshape(4, 12).T.reshape(-1).copy())
