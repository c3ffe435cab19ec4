"""Grouped SIRT steps over jobs with different geometries.

Each job's iterate after grouped steps equals the iterate of the same job run
alone with fp_sirt_step (to FP32 summation order), also with more jobs than
one grouped launch holds.
"""
import math

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


def _specs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.choice([23, 48, 64, 96, 128]))
        ny = int(rng.choice([nx, 37, 64]))
        nv = int(rng.choice([30, 45, 90, 120]))
        nd = int(2 * max(nx, ny) + rng.integers(0, 9))
        dsc = float(rng.uniform(2.0, 4.0) * max(nx, ny))
        out.append(dict(nx=nx, ny=ny, pixel=1.0, dsc=dsc, dsd=1.5 * dsc,
                        angles=2 * math.pi * np.arange(nv) / nv, n_det=nd,
                        det_width=float(rng.choice([0.8, 1.0, 1.3]))))
    return out


@pytest.mark.parametrize("count", [5, 14])
def test_grouped_steps_match_single_jobs(fp, torch_cuda, count):
    torch = torch_cuda
    specs = _specs(count, 100 + count)
    geoms = [fp.Geometry(**sp) for sp in specs]
    ys = [torch.from_numpy(phantoms.uniform((g.n_views, g.n_det), 200 + k, 0.0, 3.0)).cuda()
          for k, g in enumerate(geoms)]
    xs_multi = [torch.zeros((g.ny, g.nx), device="cuda") for g in geoms]
    works = [torch.empty_like(y) for y in ys]
    for g in geoms:
        fp.fp_sirt_prepare(g.handle)
    for _ in range(3):
        fp.fp_sirt_step_multi([(g.handle, x, y, w, 0.9) for g, x, y, w in zip(geoms, xs_multi, ys, works)])
    torch.cuda.synchronize()
    for k, (g, y) in enumerate(zip(geoms, ys)):
        x = torch.zeros((g.ny, g.nx), device="cuda")
        w = torch.empty_like(y)
        for _ in range(3):
            g.sirt_step(x, y, 0.9, w)
        a, b = xs_multi[k].double(), x.double()
        err = float((a - b).norm() / b.norm())
        assert err <= 1e-5, (k, specs[k]["nx"], specs[k]["ny"], err)


def test_grouped_step_rejects_bad_jobs(fp, torch_cuda):
    torch = torch_cuda
    g = fp.Geometry(**_specs(1, 7)[0])
    y = torch.zeros((g.n_views, g.n_det), device="cuda")
    x = torch.zeros((g.ny, g.nx), device="cuda")
    with pytest.raises(fp.FanprojError):
        fp.fp_sirt_step_multi([(g.handle, x, y, y.clone(), float("nan"))])
    fp.fp_sirt_step_multi([])  # no-op
