"""Named scan geometries and seeded input recipes.

Plain data plus calls into ``phantoms``; no projection arithmetic.  Sizes:

* ``small``  64 x 64, 90 views over 2 pi, 128 cells of width 1.5,
  source-centre 128, source-detector 256 (the CPU-fast case);
* ``medium`` 512 x 512, 720 views, 1024 cells of width 1.0, 1000 / 1500
  (the throughput workload: one forward plus one back projection);
* ``large``  2048 x 2048, 1440 views, 2048 cells of width 1.0, 4000 / 6000
  (SIRT from zero on a Poisson-noisy sinogram);
* ``fd``     32 x 32, 45 views, 64 cells of width 1.5, 64 / 128 (the small
  instance for finite-difference gradient checks).

All use the pixel size 1 and the flat detector of Sec. II-A.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import phantoms


@dataclass(frozen=True)
class Scan:
    name: str
    n: int                    # image side (nx = ny = n)
    n_views: int
    n_det: int
    det_width: float
    dsc: float                # source-to-centre distance
    dsd: float                # source-to-detector distance
    pixel: float = 1.0
    angles: np.ndarray = field(default=None, compare=False, repr=False)

    def view_angles(self) -> np.ndarray:
        return phantoms.view_angles(self.n_views) if self.angles is None else self.angles

    def kwargs(self) -> dict:
        """Arguments in the order of the geometry constructor."""
        return dict(nx=self.n, ny=self.n, pixel=self.pixel, dsc=self.dsc,
                    dsd=self.dsd, angles=self.view_angles(), n_det=self.n_det,
                    det_width=self.det_width)


SMALL = Scan("small", 64, 90, 128, 1.5, 128.0, 256.0)
MEDIUM = Scan("medium", 512, 720, 1024, 1.0, 1000.0, 1500.0)
LARGE = Scan("large", 2048, 1440, 2048, 1.0, 4000.0, 6000.0)
FD = Scan("fd", 32, 45, 64, 1.5, 64.0, 128.0)

SCANS = {s.name: s for s in (SMALL, MEDIUM, LARGE, FD)}


def phantom(scan: Scan, seed: int | None = None, count: int | None = None) -> np.ndarray:
    """The seeded ellipse phantom of a scan (float32, [n][n]).

    small: 5 ellipses, seed 1, semi-axes 4-20 px.  Larger scans: 20 ellipses
    with the semi-axis range scaled by n/64 (seed 2 for medium, 3 for large).
    """
    defaults = {"small": (1, 5), "medium": (2, 20), "large": (3, 20), "fd": (7, 3)}
    s0, c0 = defaults.get(scan.name, (0, 20))
    seed = s0 if seed is None else seed
    count = c0 if count is None else count
    scale = scan.n / 64.0
    return phantoms.ellipses(scan.n, count, seed, (4.0 * scale, 20.0 * scale), scan.pixel)


def disk_phantom(scan: Scan) -> np.ndarray:
    """Area-weighted centred unit disk: radius 200 px on medium, 24 px on small,
    3/8 of the side otherwise."""
    r = {"medium": 200.0, "small": 24.0}.get(scan.name, 0.375 * scan.n)
    return phantoms.disk(scan.n, r, scan.pixel)
