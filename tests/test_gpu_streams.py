"""The library's launch scratch is a set of per-device buffers reused across
calls and ordered on the device by events.  These tests run calls that share
those buffers in every way a caller can: back to back on one stream, on two
streams from two host threads at once, and with a buffer growing between
calls.  Every result must equal the same call made alone (the kernels are
deterministic, so bit for bit)."""
import threading

import numpy as np
import pytest

from paper_1907_10526_amd import phantoms

pytestmark = pytest.mark.gpu


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


def _geometry(fp, n, nv, seed_angle=0.0):
    angles = seed_angle + 2 * np.pi * np.arange(nv) / nv
    return fp.Geometry(n, n, 1.0, 3.0 * n, 4.5 * n, angles, 2 * n, 1.0)


def _images(torch, n, count, seed):
    return [torch.from_numpy(phantoms.uniform((n, n), seed + k, 0.0, 1.0)).float().cuda()
            for k in range(count)]


def test_two_streams_two_threads(fp, torch_cuda):
    torch = torch_cuda
    geoms = [_geometry(fp, 96, 60), _geometry(fp, 64, 45, 0.3)]
    imgs = [_images(torch, 96, 6, 10), _images(torch, 64, 6, 20)]
    # each call alone, on the default stream
    ref = [[g.back(g.forward(x)).cpu() for x in xs] for g, xs in zip(geoms, imgs)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [[None] * 6, [None] * 6]
    errors = []

    def worker(k):
        try:
            with torch.cuda.stream(streams[k]):
                for i, x in enumerate(imgs[k]):
                    out[k][i] = geoms[k].back(geoms[k].forward(x))
            streams[k].synchronize()
        except Exception as e:   # surfaced in the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k in range(2):
        for i in range(6):
            assert torch.equal(out[k][i].cpu(), ref[k][i]), (k, i)


def test_buffers_grow_between_calls(fp, torch_cuda):
    """A small call, a call needing larger scratch, then the small one again,
    queued without waiting in between."""
    torch = torch_cuda
    small, large = _geometry(fp, 48, 30), _geometry(fp, 256, 180)
    xs, xl = _images(torch, 48, 1, 30)[0], _images(torch, 256, 1, 31)[0]
    ref_s = small.back(small.forward(xs)).cpu()
    ref_l = large.back(large.forward(xl)).cpu()
    batch = torch.stack([xl] * 4)
    a = small.back(small.forward(xs))
    b = large.back(large.forward(batch))
    c = small.back(small.forward(xs))
    torch.cuda.synchronize()
    assert torch.equal(a.cpu(), ref_s) and torch.equal(c.cpu(), ref_s)
    for k in range(4):
        assert torch.equal(b[k].cpu(), ref_l), k


def test_sirt_steps_back_to_back(fp, torch_cuda):
    """SIRT steps on two geometries interleaved on one stream (each step
    takes two scratch buffers) equal the steps run geometry by geometry."""
    torch = torch_cuda
    geoms = [_geometry(fp, 64, 40), _geometry(fp, 80, 50, 0.2)]
    ys = [torch.from_numpy(phantoms.uniform((g.n_views, g.n_det), 40 + k, 0.0, 4.0)).float().cuda()
          for k, g in enumerate(geoms)]
    refs = []
    for g, y in zip(geoms, ys):
        x = torch.zeros((g.ny, g.nx), device="cuda")
        for _ in range(4):
            g.sirt_step(x, y)
        refs.append(x.cpu())
    xs = [torch.zeros((g.ny, g.nx), device="cuda") for g in geoms]
    for _ in range(4):
        for g, x, y in zip(geoms, xs, ys):
            g.sirt_step(x, y)
    torch.cuda.synchronize()
    for x, r in zip(xs, refs):
        assert torch.equal(x.cpu(), r)
