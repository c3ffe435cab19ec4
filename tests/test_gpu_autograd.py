"""Differentiation through the projector (A as a torch.autograd.Function
whose backward is the hand-written A^T kernel).

* FP64: torch.autograd.gradcheck of project/backproject on a 32 x 32,
  45-view, 64-cell instance (cell width 1.5, source-centre 64,
  source-detector 128); central finite differences of the regularised
  least-squares loss along random directions; FP64 kernels against the FP64
  oracle to 1e-10.
* FP32: the gradient of 0.5 ||A c - y||^2 against the oracle's
  A^T (A c - y) in FP64; 100 gradient steps on a batch of 16 images of the
  512 x 512 scan decrease the loss monotonically, and the batch equals the
  single-image runs.
"""
import math

import numpy as np
import pytest

from paper_1907_10526_amd import phantoms, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def mods(torch_cuda):
    from paper_1907_10526_amd import autograd, fanproj
    return fanproj, autograd


def _fd_geom(fanproj):
    s = workloads.FD
    return fanproj.Geometry(**s.kwargs()), s


def grad_sq(c, torch):
    """||grad c||^2 with forward differences and a Neumann boundary."""
    dx = c[..., :, 1:] - c[..., :, :-1]
    dy = c[..., 1:, :] - c[..., :-1, :]
    return (dx * dx).sum() + (dy * dy).sum()


def test_f64_kernels_match_oracle(oracle_mod, mods, torch_cuda):
    torch = torch_cuda
    fanproj, _ = mods
    g, s = _fd_geom(fanproj)
    og = oracle_mod.Geometry(**s.kwargs())
    c = phantoms.uniform((s.n, s.n), 51).astype(np.float64)
    y = phantoms.uniform((s.n_views, s.n_det), 52).astype(np.float64)
    yg = g.forward(torch.from_numpy(c).cuda()).cpu().numpy()
    zg = g.back(torch.from_numpy(y).cuda()).cpu().numpy()
    ey = np.linalg.norm(yg - og.forward(c)) / np.linalg.norm(og.forward(c))
    ez = np.linalg.norm(zg - og.back(y)) / np.linalg.norm(og.back(y))
    print(f"FP64 kernels vs oracle: forward {ey:.2e}, back {ez:.2e}", flush=True)
    assert ey < 1e-10 and ez < 1e-10


def test_gradcheck_f64(mods, torch_cuda):
    torch = torch_cuda
    fanproj, ag = mods
    g, s = _fd_geom(fanproj)
    c = torch.from_numpy(phantoms.uniform((s.n, s.n), 53).astype(np.float64)).cuda().requires_grad_()
    assert torch.autograd.gradcheck(lambda x: ag.project(x, g), (c,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6, fast_mode=True)
    y = torch.from_numpy(phantoms.uniform((s.n_views, s.n_det), 54).astype(np.float64)).cuda()
    y.requires_grad_()
    assert torch.autograd.gradcheck(lambda x: ag.backproject(x, g), (y,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6, fast_mode=True)


def test_loss_finite_differences_f64(mods, torch_cuda):
    torch = torch_cuda
    fanproj, ag = mods
    g, s = _fd_geom(fanproj)
    y = torch.from_numpy(phantoms.uniform((s.n_views, s.n_det), 55, 0.0, 3.0).astype(np.float64)).cuda()
    c = torch.from_numpy(phantoms.uniform((s.n, s.n), 56, 0.0, 1.0).astype(np.float64)).cuda()

    def loss(x):
        r = ag.project(x, g) - y
        return 0.5 * (r * r).sum() + 1e-3 * grad_sq(x, torch)

    x = c.clone().requires_grad_()
    loss(x).backward()
    grad = x.grad.detach()
    rng = np.random.default_rng(57)
    h = 1e-4
    for _ in range(4):
        d = torch.from_numpy(rng.standard_normal((s.n, s.n))).cuda()
        with torch.no_grad():
            fd = (loss(c + h * d) - loss(c - h * d)) / (2 * h)
        an = float((grad * d).sum())
        assert abs(float(fd) - an) <= 1e-7 * max(1.0, abs(an)), (float(fd), an)


def test_gradient_f32_matches_oracle_adjoint(oracle_mod, mods, torch_cuda):
    torch = torch_cuda
    fanproj, ag = mods
    s = workloads.SMALL
    g = fanproj.Geometry(**s.kwargs())
    og = oracle_mod.Geometry(**s.kwargs())
    c = workloads.phantom(s)
    y = phantoms.uniform((s.n_views, s.n_det), 58, 0.0, 5.0)
    x = torch.from_numpy(c).cuda().requires_grad_()
    r = ag.project(x, g) - torch.from_numpy(y).cuda()
    (0.5 * (r * r).sum()).backward()
    ref = og.back(og.forward(c.astype(np.float64)) - y.astype(np.float64))
    err = np.linalg.norm(x.grad.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"FP32 gradient vs oracle adjoint rel-L2 {err:.2e}", flush=True)
    assert err <= 1e-5


def test_batch16_gradient_descent(mods, torch_cuda):
    """Sixteen 512 x 512 phantoms, shared 720-view geometry: 100 steps of
    gradient descent on 0.5 ||A c - y||^2 + 1e-3 ||grad c||^2 with step
    1 / (||A||^2 + 16e-3) (||A||^2 from 20 power iterations)."""
    torch = torch_cuda
    fanproj, ag = mods
    s = workloads.MEDIUM
    g = fanproj.Geometry(**s.kwargs())
    truth = torch.from_numpy(np.stack([workloads.phantom(s, seed=400 + k) for k in range(16)])).cuda()
    with torch.no_grad():
        y = g.forward(truth)
    lam = ag.power_norm_sq(g, iters=20)
    step = 1.0 / (lam + 16e-3)

    def loss_fn(x):
        r = ag.project(x, g) - y
        per = 0.5 * (r * r).sum(dim=(1, 2)) + 1e-3 * torch.stack([grad_sq(x[k], torch) for k in range(x.shape[0])])
        return per

    x = torch.zeros_like(truth, requires_grad=True)
    losses = []
    for it in range(100):
        per = loss_fn(x)
        total = per.sum()
        x.grad = None
        total.backward()
        with torch.no_grad():
            x -= step * x.grad
        losses.append(float(total))
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 0.2 * losses[0]
    # the batch of 16 equals single-image runs of the same arithmetic
    with torch.no_grad():
        yb = g.forward(x.detach())
        for k in (0, 7, 15):
            assert torch.equal(yb[k], g.forward(x.detach()[k].contiguous()))
