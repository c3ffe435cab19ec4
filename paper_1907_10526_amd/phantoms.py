"""Seeded synthetic inputs: ellipse phantoms, a uniform disk, noise.

This module holds no projection arithmetic: it only draws images and
sinograms that the tests, the benchmark and the examples feed to both the GPU
library and the FP64 oracle.  Every generator is a pure function of its seed
(numpy's PCG64 through ``numpy.random.default_rng``).

The paper's phantoms (Shepp-Logan, a brain slice; Sec. V-B, V-D) are not
available here; random ellipses of the same kind of piecewise-constant
structure stand in for them.
"""
from __future__ import annotations

import numpy as np


def view_angles(n_views: int) -> np.ndarray:
    """n_views angles uniformly spaced over [0, 2 pi), endpoint excluded."""
    return 2.0 * np.pi * np.arange(n_views, dtype=np.float64) / n_views


def pixel_centres(n: int, pixel: float = 1.0):
    """x (columns) and y (rows) of the centres of an n x n grid centred on 0."""
    c = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * pixel
    return np.meshgrid(c, c, indexing="xy")  # X[j, i] = x_i, Y[j, i] = y_j


def ellipse_params(n: int, count: int, seed: int, semi_axes_px=(4.0, 20.0),
                   pixel: float = 1.0) -> np.ndarray:
    """Parameters of `count` random ellipses, one row each:
    (cx, cy, semi-axis a, semi-axis b, orientation, intensity).

    Centres are uniform in the disk of radius n/2 pixels (rho = sqrt(U),
    phi = 2 pi U); semi-axes are uniform in `semi_axes_px` (pixels);
    orientation is uniform in [0, pi); intensity is uniform in [-0.5, 1].
    """
    rng = np.random.default_rng(seed)
    rho = np.sqrt(rng.random(count))
    phi = 2.0 * np.pi * rng.random(count)
    lo, hi = semi_axes_px
    a = rng.uniform(lo, hi, count)
    b = rng.uniform(lo, hi, count)
    ang = rng.uniform(0.0, np.pi, count)
    val = rng.uniform(-0.5, 1.0, count)
    r = 0.5 * n * pixel * rho
    return np.stack([r * np.cos(phi), r * np.sin(phi), a * pixel, b * pixel, ang, val], axis=1)


def ellipses(n: int, count: int, seed: int, semi_axes_px=(4.0, 20.0),
             pixel: float = 1.0, dtype=np.float32) -> np.ndarray:
    """n x n image of random ellipses, rasterised by sampling at pixel
    centres; overlapping ellipses add.  Row j holds y_j, column i holds x_i."""
    X, Y = pixel_centres(n, pixel)
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, ang, val in ellipse_params(n, count, seed, semi_axes_px, pixel):
        c, s = np.cos(ang), np.sin(ang)
        dx, dy = X - cx, Y - cy
        xr = c * dx + s * dy
        yr = -s * dx + c * dy
        img += val * ((xr / a) ** 2 + (yr / b) ** 2 <= 1.0)
    return img.astype(dtype)


def disk(n: int, radius_px: float, pixel: float = 1.0, value: float = 1.0,
         supersample: int = 16, dtype=np.float32) -> np.ndarray:
    """Centred uniform disk, each pixel weighted by the fraction of its area
    inside the disk (supersample x supersample point samples per pixel)."""
    r = radius_px * pixel
    sub = (np.arange(supersample, dtype=np.float64) + 0.5) / supersample - 0.5
    c = (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * pixel
    xs = (c[:, None] + sub[None, :] * pixel).reshape(-1)  # n*ss positions
    inside_x = xs[None, :] ** 2  # (1, n*ss)
    img = np.zeros((n, n), dtype=np.float64)
    for j in range(n):
        ys = c[j] + sub * pixel
        hit = (inside_x + ys[:, None] ** 2) <= r * r  # (ss, n*ss)
        img[j] = hit.reshape(supersample, n, supersample).mean(axis=(0, 2))
    return (value * img).astype(dtype)


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0, dtype=np.float32):
    """Seeded i.i.d. uniform array (for adjoint identities and random probes)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(dtype)


def poisson_log_sinogram(clean_sino: np.ndarray, i0: float, seed: int,
                         dtype=np.float32) -> np.ndarray:
    """Noisy line integrals: counts N ~ Poisson(i0 exp(-y)), y_noisy =
    ln(i0 / max(N, 1))."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(i0 * np.exp(-np.asarray(clean_sino, dtype=np.float64)))
    return np.log(i0 / np.maximum(counts, 1)).astype(dtype)
