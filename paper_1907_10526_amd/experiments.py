"""The paper's experiments that need no datasets (Sec. V), run on the GPU.

Each function returns plain numbers (JSON-ready).  Geometry values are the
paper's: its D_po is the source-centre distance here and D_po + D_so the
source-detector distance; its Shepp-Logan and brain phantoms are replaced by
seeded non-negative ellipse phantoms of the same sizes.

* ``single_pixel``   (Sec. V-A, first experiment): one 1 x 1 pixel at the
  centre, D_po = D_so = 3, cell width 0.5, cell pitch 0.01, 601 cells; the
  CNSF projection against the reference at 0, 15, 35 and 45 degrees.
* ``max_error``      (Sec. V-A, e(u)): the maximum over cells of
  |CNSF - Ref| for one pixel at (0, 0) (90 angles over 90 degrees) and at
  (100.5, 50.5) (360 angles), width = pitch = 0.5, D_po = D_so = 200.
* ``image_error``    (Sec. V-B): sinogram-domain errors of CNSF against the
  reference for a 128 x 128 image (409 cells, D_po = D_so = 200) and a
  256 x 256 image (815 cells, D_po = D_so = 400), pitch 1, width 0.5,
  360 views.
* ``timing``         (Sec. V-C): forward and back projection times of
  all-ones images from 64 x 64 to 2048 x 2048 with the paper's detector counts
  and distances, 360 views, width = pitch = 1.
* ``reconstruction`` (Sec. V-D): data from the reference projector,
  reconstructed by SIRT with the reference operators and with CNSF; SNR of
  each against the phantom (128 x 128 from 16 views, 256 x 256 from 30 views).

    python -m paper_1907_10526_amd.experiments [--which NAME ...] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import phantoms

__all__ = ["single_pixel", "max_error", "image_error", "timing", "reconstruction", "run"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the experiments run on a GPU")
    return torch


def _geom(n, dsc, dsd, angles, n_det, width, pitch=None, beam="flat", ny=None):
    from .fanproj import Geometry
    return Geometry(n, n if ny is None else ny, 1.0, dsc, dsd, angles, n_det, width, beam=beam,
                    det_pitch=pitch)


def _onehot(torch, n, i, j, ny=None):
    c = torch.zeros((n if ny is None else ny, n), dtype=torch.float64, device="cuda")
    c[j, i] = 1.0
    return c


def _phantom(n, seed):
    scale = n / 64.0
    c = phantoms.ellipses(n, 12, seed, (4.0 * scale, 16.0 * scale)).astype(np.float64)
    return np.clip(c, 0.0, None)


def single_pixel(beam="flat"):
    torch = _torch()
    degs = [0.0, 15.0, 35.0, 45.0]
    g = _geom(1, 3.0, 6.0, np.radians(degs), 601, 0.5, pitch=0.01, beam=beam)
    c = _onehot(torch, 1, 0, 0)
    y = g.forward(c).cpu().numpy()
    r = g.forward_reference(c).cpu().numpy()
    out = []
    for k, d in enumerate(degs):
        out.append({"angle_deg": d, "max_abs_err": float(np.abs(y[k] - r[k]).max()),
                    "ref_peak": float(r[k].max()),
                    "rel_l2": float(np.linalg.norm(y[k] - r[k]) / np.linalg.norm(r[k]))})
    g.close()
    return {"geometry": "1x1 pixel at the centre, D_po = D_so = 3, width 0.5, pitch 0.01, 601 cells",
            "beam": beam, "angles": out}


def max_error(beam="flat"):
    torch = _torch()
    res = {}
    # pixel at (0, 0): a 1 x 1 image; 90 angles over 90 degrees
    ang = np.arange(90) * (0.5 * math.pi / 90)
    g = _geom(1, 200.0, 400.0, ang, 64, 0.5, pitch=0.5, beam=beam)
    c = _onehot(torch, 1, 0, 0)
    e = (g.forward(c) - g.forward_reference(c)).abs().amax(dim=1).cpu().numpy()
    g.close()
    res["pixel_0_0"] = {"angles": 90, "max": float(e.max()), "mean": float(e.mean()),
                        "e_per_angle": [float(x) for x in e]}
    # pixel at (100.5, 50.5): the last pixel (201, 101) of a 202 x 102 grid
    # centred on the rotation centre; 360 angles
    ang = np.arange(360) * (2 * math.pi / 360)
    g = _geom(202, 200.0, 400.0, ang, 2200, 0.5, pitch=0.5, beam=beam, ny=102)
    c = _onehot(torch, 202, 201, 101, ny=102)
    e = (g.forward(c) - g.forward_reference(c)).abs().amax(dim=1).cpu().numpy()
    g.close()
    res["pixel_100.5_50.5"] = {"angles": 360, "max": float(e.max()), "mean": float(e.mean()),
                               "e_per_angle": [float(x) for x in e]}
    return {"geometry": "width = pitch = 0.5, D_po = D_so = 200", "beam": beam, **res}


def image_error(beam="flat"):
    torch = _torch()
    out = []
    for n, nd, dpo, seed in [(128, 409, 200.0, 71), (256, 815, 400.0, 72)]:
        ang = np.arange(360) * (2 * math.pi / 360)
        g = _geom(n, dpo, 2 * dpo, ang, nd, 0.5, pitch=1.0, beam=beam)
        c = torch.from_numpy(_phantom(n, seed)).cuda()
        y = g.forward(c)
        r = g.forward_reference(c)
        d = (y - r).abs()
        out.append({"image": n, "cells": nd, "D_po": dpo, "max_abs_err": float(d.max()),
                    "mean_abs_err": float(d.mean()), "ref_max": float(r.abs().max()),
                    "rel_l2": float((y - r).norm() / r.norm())})
        g.close()
    return {"geometry": "pitch 1, width 0.5, 360 views, D_so = D_po", "beam": beam,
            "phantom": "12 seeded non-negative ellipses", "images": out}


def timing(reps=10):
    torch = _torch()
    rows = []
    for n, nd, dpo in [(64, 205, 100.0), (128, 409, 200.0), (256, 815, 400.0), (512, 1627, 800.0),
                       (1024, 3250, 1600.0), (2048, 6499, 3200.0)]:
        ang = np.arange(360) * (2 * math.pi / 360)
        g = _geom(n, dpo, 2 * dpo, ang, nd, 1.0)
        c = torch.ones((n, n), device="cuda")
        y = g.forward(c)
        z = g.back(y)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(reps):
            g.forward(c, out=y)
        ev[1].record()
        for _ in range(reps):
            g.back(y, out=z)
        ev[2].record()
        torch.cuda.synchronize()
        f = ev[0].elapsed_time(ev[1]) / reps
        b = ev[1].elapsed_time(ev[2]) / reps
        nnz = g.count_nonzero()
        rows.append({"image": n, "cells": nd, "D_po": dpo, "forward_ms": f, "back_ms": b,
                     "forward_ms_per_view": f / 360, "back_ms_per_view": b / 360,
                     "nonzero_entries": nnz,
                     "entries_per_s": {"forward": nnz / (f * 1e-3), "back": nnz / (b * 1e-3)}})
        g.close()
    return {"geometry": "360 views, width = pitch = 1, D_so = D_po, all-ones images, FP32",
            "sizes": rows}


def _snr(x, ref):
    return float(10.0 * np.log10(np.sum(ref * ref) / np.sum((x - ref) ** 2)))


def _sirt(torch, fwd, back, y, shape, iters):
    ones_img = torch.ones(shape, dtype=torch.float64, device="cuda")
    rs = fwd(ones_img)
    cs = back(torch.ones_like(y))
    R = torch.where(rs != 0, 1.0 / rs, torch.zeros_like(rs))
    C = torch.where(cs != 0, 1.0 / cs, torch.zeros_like(cs))
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    for _ in range(iters):
        x = x + C * back(R * (y - fwd(x)))
    return x


RECONSTRUCTION_RUNS = ((128, 409, 200.0, 16, 81), (256, 815, 400.0, 30, 82))


def reconstruction(iters=300, beam="flat", runs=RECONSTRUCTION_RUNS):
    """runs: (image size, cells, D_po, views, phantom seed) per reconstruction."""
    torch = _torch()
    out = []
    for n, nd, dpo, nv, seed in runs:
        ang = np.arange(nv) * (2 * math.pi / nv)
        g = _geom(n, dpo, 2 * dpo, ang, nd, 1.0, pitch=1.0, beam=beam)
        truth = _phantom(n, seed)
        y = g.forward_reference(torch.from_numpy(truth).cuda())
        t0 = time.perf_counter()
        x_ref = _sirt(torch, g.forward_reference, g.back_reference, y, (n, n), iters).cpu().numpy()
        t1 = time.perf_counter()
        x_cnsf = _sirt(torch, g.forward, g.back, y, (n, n), iters).cpu().numpy()
        t2 = time.perf_counter()
        out.append({"image": n, "views": nv, "cells": nd, "D_po": dpo, "iterations": iters,
                    "snr_db": {"ref": _snr(x_ref, truth), "cnsf": _snr(x_cnsf, truth)},
                    "cnsf_minus_ref_rel_l2": float(np.linalg.norm(x_cnsf - x_ref) / np.linalg.norm(x_ref)),
                    "seconds": {"ref": t1 - t0, "cnsf": t2 - t1}})
        g.close()
    return {"data": "reference projector, noise-free", "solver": "SIRT from zero, FP64",
            "beam": beam, "phantom": "12 seeded non-negative ellipses", "runs": out}


EXPERIMENTS = {"single_pixel": single_pixel, "max_error": max_error, "image_error": image_error,
               "timing": timing, "reconstruction": reconstruction}


def run(which=None, progress=print):
    res = {}
    for name in which or list(EXPERIMENTS):
        t0 = time.perf_counter()
        res[name] = EXPERIMENTS[name]()
        progress(f"{name} done in {time.perf_counter() - t0:.1f} s", flush=True)
    return res


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--which", nargs="*", choices=list(EXPERIMENTS), default=None)
    p.add_argument("--out", default=None, help="write the JSON results here")
    args = p.parse_args()
    res = run(args.which)
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
