"""FP64 CPU oracle for the CNSF fan-beam projector (arXiv 1907.10526).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product package never
does, and the oracle imports nothing from the product package.

The arithmetic lives in ``cnsf_oracle.c`` (plain C, double precision, OpenMP
loops).  This module builds it with gcc into ``libcnsf_oracle.so`` next to the
source and wraps it with ctypes; arrays are numpy float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cnsf_oracle.c")
_LIB = os.path.join(_HERE, "libcnsf_oracle.so")

FAN_FLAT = 0
PARALLEL = 1
FAN_ARC = 2


def build(force: bool = True) -> str:
    """Compile the oracle into a shared library (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("pixel", ctypes.c_double),
        ("dsc", ctypes.c_double), ("dsd", ctypes.c_double),
        ("n_views", ctypes.c_int32),
        ("angles", ctypes.POINTER(ctypes.c_double)),
        ("n_det", ctypes.c_int32),
        ("det_spacing", ctypes.c_double), ("det_width", ctypes.c_double),
        ("mode", ctypes.c_int32),
    ]


_dll = None


def _lib():
    global _dll
    if _dll is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        d = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Geom)
        dp = ctypes.POINTER(ctypes.c_double)
        d.oracle_box3.argtypes = [ctypes.c_double] * 4
        d.oracle_box3.restype = ctypes.c_double
        d.oracle_box2.argtypes = [ctypes.c_double] * 3
        d.oracle_box2.restype = ctypes.c_double
        d.oracle_entry.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        d.oracle_entry.restype = ctypes.c_double
        d.oracle_entry_terms.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         dp, dp, dp, dp, dp]
        d.oracle_entry_terms.restype = None
        d.oracle_forward.argtypes = [P, dp, dp, ctypes.c_int]
        d.oracle_back.argtypes = [P, dp, dp, ctypes.c_int]
        d.oracle_forward_cached.argtypes = [P, dp, dp]
        d.oracle_forward_cached.restype = ctypes.c_int
        d.oracle_back_cached.argtypes = [P, dp, dp]
        d.oracle_back_cached.restype = ctypes.c_int
        d.oracle_forward_ray.argtypes = [P, dp, ctypes.c_int, ctypes.c_int]
        d.oracle_forward_ray.restype = ctypes.c_double
        d.oracle_back_pixel.argtypes = [P, dp, ctypes.c_int, ctypes.c_int]
        d.oracle_back_pixel.restype = ctypes.c_double
        d.oracle_forward_views.argtypes = [P, dp, dp, ctypes.c_int, ctypes.c_int]
        d.oracle_back_views.argtypes = [P, dp, dp, ctypes.c_int, ctypes.c_int]
        d.oracle_count_nonzero.argtypes = [P]
        d.oracle_count_nonzero.restype = ctypes.c_int64
        d.oracle_sirt.argtypes = [P, dp, dp, ctypes.c_int, ctypes.c_double]
        d.oracle_threads.restype = ctypes.c_int
        d.oracle_set_threads.argtypes = [ctypes.c_int]
        _dll = d
    return _dll


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def box3(x, w1, w2, w3) -> float:
    """Centred unit-mass 3-direction box spline M_[w1,w2,w3](x) (eq. (9), (18))."""
    return _lib().oracle_box3(float(x), float(w1), float(w2), float(w3))


def box2(x, w1, w2) -> float:
    """Centred unit-mass 2-direction box spline M_[w1,w2](x) (eq. (16))."""
    return _lib().oracle_box2(float(x), float(w1), float(w2))


def set_threads(n: int) -> None:
    _lib().oracle_set_threads(int(n))


def threads() -> int:
    return _lib().oracle_threads()


class Geometry:
    """Fan-beam (flat or arc detector) or parallel-beam scan description.

    Pixel (i, j) is centred at ((i-(nx-1)/2) delta, (j-(ny-1)/2) delta); cell m
    at s_m = (m-(n_det-1)/2) * det_spacing on the detector axis
    (sin t, -cos t); the source of view t sits at dsc * (cos t, sin t) and the
    flat detector is perpendicular to that direction at distance dsd from the
    source (Sec. II-A).  With mode=FAN_ARC the cells lie on the circle of
    radius dsd around the source and s is arc length on it; with
    mode=PARALLEL every ray of a view runs along -(cos t, sin t).
    """

    def __init__(self, nx, ny, pixel, dsc, dsd, angles, n_det, det_width,
                 det_spacing=None, mode=FAN_FLAT):
        self.nx, self.ny = int(nx), int(ny)
        self.pixel = float(pixel)
        self.dsc, self.dsd = float(dsc), float(dsd)
        self.angles = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
        self.n_views = int(self.angles.size)
        self.n_det = int(n_det)
        self.det_width = float(det_width)
        self.det_spacing = float(det_width if det_spacing is None else det_spacing)
        self.mode = int(mode)
        self._c = _Geom(self.nx, self.ny, self.pixel, self.dsc, self.dsd,
                        self.n_views, _dptr(self.angles), self.n_det,
                        self.det_spacing, self.det_width, self.mode)

    @property
    def _p(self):
        return ctypes.byref(self._c)

    # -- single entries -------------------------------------------------
    def entry(self, v, m, i, j) -> float:
        """A_{(v,m),(i,j)} = delta^2 M_[zeta1, zeta2, tau'](s')  (eq. (18))."""
        return _lib().oracle_entry(self._p, int(v), int(m), int(i), int(j))

    def entry_terms(self, v, m, i, j):
        """(s', zeta1, zeta2, tau', L) of eq. (13), (16), (17)."""
        out = [ctypes.c_double() for _ in range(5)]
        _lib().oracle_entry_terms(self._p, int(v), int(m), int(i), int(j),
                                  *[ctypes.byref(o) for o in out])
        return tuple(o.value for o in out)

    # -- operators --------------------------------------------------------
    def forward(self, img, dense=False, cached=False) -> np.ndarray:
        """A c.  dense: every (ray, pixel) pair; cached: the same pruned sums
        with the ray frames computed once (bitwise equal to the default)."""
        img = np.ascontiguousarray(img, dtype=np.float64).reshape(self.ny, self.nx)
        out = np.empty((self.n_views, self.n_det), dtype=np.float64)
        if cached and not dense:
            if _lib().oracle_forward_cached(self._p, _dptr(img), _dptr(out)) != 0:
                raise MemoryError("oracle_forward_cached: frame table allocation failed")
        else:
            _lib().oracle_forward(self._p, _dptr(img), _dptr(out), int(bool(dense)))
        return out

    def back(self, sino, dense=False, cached=False) -> np.ndarray:
        """A^T y, with the same options as forward."""
        sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(self.n_views, self.n_det)
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        if cached and not dense:
            if _lib().oracle_back_cached(self._p, _dptr(sino), _dptr(out)) != 0:
                raise MemoryError("oracle_back_cached: frame table allocation failed")
        else:
            _lib().oracle_back(self._p, _dptr(sino), _dptr(out), int(bool(dense)))
        return out

    def forward_ray(self, img, v, m) -> float:
        img = np.ascontiguousarray(img, dtype=np.float64).reshape(self.ny, self.nx)
        return _lib().oracle_forward_ray(self._p, _dptr(img), int(v), int(m))

    def back_pixel(self, sino, i, j) -> float:
        sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(self.n_views, self.n_det)
        return _lib().oracle_back_pixel(self._p, _dptr(sino), int(i), int(j))

    def forward_views(self, img, v0, v1) -> np.ndarray:
        """Rows v0..v1-1 of A c (other rows are left zero)."""
        img = np.ascontiguousarray(img, dtype=np.float64).reshape(self.ny, self.nx)
        out = np.zeros((self.n_views, self.n_det), dtype=np.float64)
        _lib().oracle_forward_views(self._p, _dptr(img), _dptr(out), int(v0), int(v1))
        return out

    def back_views(self, sino, v0, v1) -> np.ndarray:
        """A^T y summed over views v0..v1-1 only."""
        sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(self.n_views, self.n_det)
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        _lib().oracle_back_views(self._p, _dptr(sino), _dptr(out), int(v0), int(v1))
        return out

    def count_nonzero(self) -> int:
        return int(_lib().oracle_count_nonzero(self._p))

    def sirt(self, y, iters, x0=None, relaxation=1.0) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(self.n_views, self.n_det)
        x = (np.zeros((self.ny, self.nx)) if x0 is None
             else np.array(x0, dtype=np.float64).reshape(self.ny, self.nx))
        x = np.ascontiguousarray(x)
        _lib().oracle_sirt(self._p, _dptr(y), _dptr(x), int(iters), float(relaxation))
        return x
