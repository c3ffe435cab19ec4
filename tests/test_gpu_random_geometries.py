"""Seeded sweeps of random small geometries against the FP64 oracle.

Each case draws the beam shape, image size, pixel size, cell count, cell
width and pitch, distances and view angles, so that the kernels' window
sizing (per-block widths in the forward walk, per-tile windows in the back
projection), the fixed-point row stepping and the edge clamps meet many
combinations the hand-picked tests do not.  A second sweep draws square
scans whose views repeat under quarter turns, with and without the diagonal
reflection, so that the symmetric forms (symmetry order 8 and 4) meet random
sizes, pitches and distances as well.  Bar: relative L2 error <= 1e-5 for
forward and back projection, dense oracle (every ray-pixel pair)."""
import math

import numpy as np
import pytest

from paper_1907_10526_amd import phantoms

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


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    beam = ["flat", "arc", "parallel"][seed % 3]
    nx, ny = (int(v) for v in rng.integers(4, 49, size=2))
    pixel = float(rng.uniform(0.5, 2.0))
    width = pixel * float(rng.uniform(0.3, 2.0))
    pitch = width * float(rng.uniform(0.8, 1.5))
    half_diag = pixel * (0.5 * math.hypot(nx, ny) + 1.0)
    dsc = half_diag * float(rng.uniform(1.05, 6.0))
    dsd = dsc * float(rng.uniform(1.1, 3.0))
    # enough cells to cover the image's shadow, plus some that miss it; cells
    # no narrower than an eighth of a magnified pixel, so that a 16 x 32 tile
    # spans a few hundred cells at most (the on-chip staging limit)
    mag = 1.0 if beam == "parallel" else dsd / max(dsc - half_diag, 1e-3)
    pitch = max(pitch, pixel * mag / 8.0)
    nd = int(min(max(2.0 * half_diag * mag / pitch * float(rng.uniform(0.6, 1.4)), 3), 160))
    if beam == "arc":   # the arc detector stays within 80 degrees of the central ray
        nd = int(min(nd, (1.39 * dsd - 0.5 * width) / pitch * 2.0 - 1.0))
    nv = int(rng.integers(3, 41))
    angles = rng.uniform(0.0, 2.0 * math.pi, nv)
    kw = dict(nx=nx, ny=ny, pixel=pixel, dsc=dsc, dsd=dsd, angles=angles, n_det=max(nd, 1),
              det_width=width)
    return beam, pitch, kw


@pytest.mark.parametrize("seed", range(24))
def test_random_geometry(oracle_mod, fp, torch_cuda, seed):
    torch = torch_cuda
    beam, pitch, kw = random_case(seed)
    og = oracle_mod.Geometry(**kw, det_spacing=pitch, mode=MODES[beam])
    gg = fp.Geometry(**kw, beam=beam, det_pitch=pitch)
    label = (f"case {seed}: {beam} {kw['nx']}x{kw['ny']} pixel {kw['pixel']:.3f} "
             f"views {len(kw['angles'])} cells {kw['n_det']} width {kw['det_width']:.3f} "
             f"pitch {pitch:.3f} dsc {kw['dsc']:.2f} dsd {kw['dsd']:.2f}")
    print(label, flush=True)
    img = phantoms.uniform((gg.ny, gg.nx), seed, 0.0, 1.0)
    y = gg.forward(torch.from_numpy(img).cuda()).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    sino = phantoms.uniform((gg.n_views, gg.n_det), seed + 100, 0.0, 1.0)
    z = gg.back(torch.from_numpy(sino).cuda()).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    if np.linalg.norm(y_ref) == 0.0:   # every ray misses the image
        assert np.all(y == 0.0) and np.all(z == 0.0)
        return
    ef, eb = rel_l2(y, y_ref), rel_l2(z, z_ref)
    print(f"  forward rel-L2 {ef:.3e}, back rel-L2 {eb:.3e}", flush=True)
    assert ef <= TOL and eb <= TOL, (label, ef, eb)


def random_symmetric_case(seed):
    """A square image with views uniform over 2 pi: from angle 0 with V a
    multiple of 8 (symmetry order 8: quarter-turn forward, octant back), or
    V a multiple of 4 off the reflection (order 4: quarter-turn forms)."""
    beam, pitch, kw = random_case(50 + seed)
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(4, 49))
    kw["nx"] = kw["ny"] = n
    half_diag = kw["pixel"] * (0.5 * math.hypot(n, n) + 1.0)
    # (source at least 1.5 half-diagonals out: magnifications that keep a
    # back-projection tile's cells within the eight-image staging)
    kw["dsc"] = max(kw["dsc"], half_diag * 1.5)
    kw["dsd"] = max(kw["dsd"], kw["dsc"] * 1.1)
    if seed % 2 == 0:
        nv, offset, order = 8 * int(rng.integers(1, 7)), 0.0, 8
    else:
        nv, offset, order = 4 * int(rng.integers(1, 11)), float(rng.uniform(0.01, 1.5)), 4
    kw["angles"] = 2.0 * math.pi * np.arange(nv) / nv + offset
    return beam, pitch, kw, order


@pytest.mark.parametrize("seed", range(16))
def test_random_symmetric_geometry(oracle_mod, fp, torch_cuda, seed):
    torch = torch_cuda
    beam, pitch, kw, order = random_symmetric_case(seed)
    og = oracle_mod.Geometry(**kw, det_spacing=pitch, mode=MODES[beam])
    gg = fp.Geometry(**kw, beam=beam, det_pitch=pitch)
    label = (f"symmetric case {seed}: {beam} {kw['nx']}^2 pixel {kw['pixel']:.3f} "
             f"views {len(kw['angles'])} cells {kw['n_det']} width {kw['det_width']:.3f} "
             f"pitch {pitch:.3f} dsc {kw['dsc']:.2f} dsd {kw['dsd']:.2f} order {gg.symmetry()}")
    print(label, flush=True)
    assert gg.symmetry() == order
    img = phantoms.uniform((gg.ny, gg.nx), 300 + seed, 0.0, 1.0)
    y = gg.forward(torch.from_numpy(img).cuda()).cpu().numpy()
    y_ref = og.forward(img.astype(np.float64), dense=True)
    sino = phantoms.uniform((gg.n_views, gg.n_det), 400 + seed, 0.0, 1.0)
    z = gg.back(torch.from_numpy(sino).cuda()).cpu().numpy()
    z_ref = og.back(sino.astype(np.float64), dense=True)
    if np.linalg.norm(y_ref) == 0.0:   # every ray misses the image
        assert np.all(y == 0.0) and np.all(z == 0.0)
        return
    ef, eb = rel_l2(y, y_ref), rel_l2(z, z_ref)
    print(f"  forward rel-L2 {ef:.3e}, back rel-L2 {eb:.3e}", flush=True)
    assert ef <= TOL and eb <= TOL, (label, ef, eb)
