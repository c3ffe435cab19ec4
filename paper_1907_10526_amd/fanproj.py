"""ctypes binding of libfanproj (the C ABI in ``include/fanproj.h``).

Argument marshalling only: every step of a projection runs in the HIP
kernels of the shared library.  Tensors are torch CUDA (HIP) float32 tensors,
passed by device pointer together with torch's current stream.  If the
library has not been built, importing this module raises ImportError; there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfanproj.so")

FP_OK = 0
FP_ERR_INVALID_ARG = 1
FP_ERR_OUT_OF_MEMORY = 2
FP_ERR_DEVICE = 3
FP_ERR_UNSUPPORTED = 4

FP_FAN_FLAT = 0
FP_FAN_ARC = 1
FP_PARALLEL = 2
BEAMS = {"flat": FP_FAN_FLAT, "arc": FP_FAN_ARC, "parallel": FP_PARALLEL}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python -m paper_1907_10526_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_lib.fp_geometry_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_vp)]
_lib.fp_geometry_create.restype = ctypes.c_int
class FpGeometryDesc(ctypes.Structure):
    """fp_geometry_desc of the C ABI."""
    _fields_ = [("beam", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("pixel_size", ctypes.c_double), ("dist_source_center", ctypes.c_double),
                ("dist_source_detector", ctypes.c_double), ("n_views", ctypes.c_int32),
                ("view_angles", ctypes.POINTER(ctypes.c_double)), ("n_det", ctypes.c_int32),
                ("det_pitch", ctypes.c_double), ("det_width", ctypes.c_double)]


_lib.fp_geometry_create_desc.argtypes = [ctypes.POINTER(FpGeometryDesc), ctypes.POINTER(_vp)]
_lib.fp_geometry_create_desc.restype = ctypes.c_int
_lib.fp_geometry_destroy.argtypes = [_vp]
_lib.fp_geometry_destroy.restype = ctypes.c_int
_lib.fp_forward.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp]
_lib.fp_forward.restype = ctypes.c_int
_lib.fp_back.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp]
_lib.fp_back.restype = ctypes.c_int
_lib.fp_forward_f64.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp]
_lib.fp_forward_f64.restype = ctypes.c_int
_lib.fp_back_f64.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp]
_lib.fp_back_f64.restype = ctypes.c_int
_lib.fp_forward_reference.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp]
_lib.fp_forward_reference.restype = ctypes.c_int
_lib.fp_back_reference.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp]
_lib.fp_back_reference.restype = ctypes.c_int
_lib.fp_sirt_step.argtypes = [_vp, _vp, _vp, ctypes.c_float, _vp, ctypes.c_int32, _vp]
_lib.fp_sirt_step.restype = ctypes.c_int
_lib.fp_sirt_step_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_float, _vp, ctypes.c_int32, _vp]
_lib.fp_sirt_step_noalloc.restype = ctypes.c_int
class FpSirtJob(ctypes.Structure):
    """fp_sirt_job of the C ABI."""
    _fields_ = [("geometry", ctypes.c_void_p), ("image", ctypes.c_void_p),
                ("sino_meas", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("relaxation", ctypes.c_float)]


_lib.fp_sirt_prepare.argtypes = [_vp, _vp]
_lib.fp_sirt_prepare.restype = ctypes.c_int
_lib.fp_sirt_step_multi.argtypes = [ctypes.POINTER(FpSirtJob), ctypes.c_int32, _vp]
_lib.fp_sirt_step_multi.restype = ctypes.c_int
_lib.fp_count_nonzero.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), _vp]
_lib.fp_count_nonzero.restype = ctypes.c_int
_lib.fp_geometry_device_bytes.argtypes = [_vp]
_lib.fp_geometry_device_bytes.restype = ctypes.c_size_t
_lib.fp_sirt_scratch_bytes.argtypes = [_vp, ctypes.c_int32]
_lib.fp_sirt_scratch_bytes.restype = ctypes.c_size_t
_lib.fp_geometry_quarter_turn.argtypes = [_vp]
_lib.fp_geometry_quarter_turn.restype = ctypes.c_int32
_lib.fp_geometry_symmetry.argtypes = [_vp]
_lib.fp_geometry_symmetry.restype = ctypes.c_int32
_lib.fp_last_error.argtypes = []
_lib.fp_last_error.restype = ctypes.c_char_p

EXPORTED = ("fp_geometry_create", "fp_geometry_create_desc", "fp_geometry_destroy", "fp_forward", "fp_back", "fp_forward_f64",
            "fp_back_f64", "fp_forward_reference", "fp_back_reference", "fp_sirt_step", "fp_sirt_step_noalloc",
            "fp_sirt_prepare", "fp_sirt_step_multi",
            "fp_count_nonzero", "fp_sirt_scratch_bytes", "fp_geometry_device_bytes", "fp_geometry_quarter_turn",
            "fp_geometry_symmetry", "fp_last_error")


class FanprojError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fanproj status {status}: {message}")
        self.status = status


def fp_last_error() -> str:
    return (_lib.fp_last_error() or b"").decode()


def _check(status: int):
    if status != FP_OK:
        raise FanprojError(status, fp_last_error())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, name, shape=None, dtype=None):
    import torch
    dtype = torch.float32 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on a GPU")
    if shape is not None and tuple(t.shape[-len(shape):]) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (..., {shape})")
    return ctypes.c_void_p(t.data_ptr())


# -- the C ABI, one Python function per entry point ---------------------------

def fp_geometry_create(nx, ny, pixel_size, dist_source_center, dist_source_detector,
                       view_angles, n_det, det_width) -> ctypes.c_void_p:
    ang = np.ascontiguousarray(np.asarray(view_angles, dtype=np.float64))
    h = ctypes.c_void_p()
    _check(_lib.fp_geometry_create(int(nx), int(ny), float(pixel_size), float(dist_source_center),
                                   float(dist_source_detector), int(ang.size),
                                   ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   int(n_det), float(det_width), ctypes.byref(h)))
    return h


def fp_geometry_create_desc(beam, nx, ny, pixel_size, dist_source_center, dist_source_detector,
                            view_angles, n_det, det_pitch, det_width) -> ctypes.c_void_p:
    ang = np.ascontiguousarray(np.asarray(view_angles, dtype=np.float64))
    d = FpGeometryDesc(int(beam), int(nx), int(ny), float(pixel_size), float(dist_source_center),
                       float(dist_source_detector), int(ang.size),
                       ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n_det),
                       float(det_pitch), float(det_width))
    h = ctypes.c_void_p()
    _check(_lib.fp_geometry_create_desc(ctypes.byref(d), ctypes.byref(h)))
    return h


def fp_geometry_destroy(handle) -> None:
    _check(_lib.fp_geometry_destroy(handle))


def fp_forward(handle, image, sino, batch, stream=None) -> None:
    _check(_lib.fp_forward(handle, _dev_ptr(image, "image"), _dev_ptr(sino, "sino"), int(batch),
                           _stream_handle(stream)))


def fp_back(handle, sino, image, batch, stream=None) -> None:
    _check(_lib.fp_back(handle, _dev_ptr(sino, "sino"), _dev_ptr(image, "image"), int(batch),
                        _stream_handle(stream)))


def fp_forward_f64(handle, image, sino, batch, stream=None) -> None:
    import torch
    _check(_lib.fp_forward_f64(handle, _dev_ptr(image, "image", dtype=torch.float64),
                               _dev_ptr(sino, "sino", dtype=torch.float64), int(batch),
                               _stream_handle(stream)))


def fp_back_f64(handle, sino, image, batch, stream=None) -> None:
    import torch
    _check(_lib.fp_back_f64(handle, _dev_ptr(sino, "sino", dtype=torch.float64),
                            _dev_ptr(image, "image", dtype=torch.float64), int(batch),
                            _stream_handle(stream)))


def fp_forward_reference(handle, image, sino, batch, quad_points=0, stream=None) -> None:
    import torch
    _check(_lib.fp_forward_reference(handle, _dev_ptr(image, "image", dtype=torch.float64),
                                     _dev_ptr(sino, "sino", dtype=torch.float64), int(batch),
                                     int(quad_points), _stream_handle(stream)))


def fp_back_reference(handle, sino, image, batch, quad_points=0, stream=None) -> None:
    import torch
    _check(_lib.fp_back_reference(handle, _dev_ptr(sino, "sino", dtype=torch.float64),
                                  _dev_ptr(image, "image", dtype=torch.float64), int(batch),
                                  int(quad_points), _stream_handle(stream)))


def fp_sirt_step(handle, image, sino_meas, relaxation, work, batch, stream=None) -> None:
    _check(_lib.fp_sirt_step(handle, _dev_ptr(image, "image"), _dev_ptr(sino_meas, "sino_meas"),
                             float(relaxation), _dev_ptr(work, "work"), int(batch),
                             _stream_handle(stream)))


def fp_sirt_step_noalloc(handle, image, sino_meas, relaxation, work, batch, stream=None) -> None:
    _check(_lib.fp_sirt_step_noalloc(handle, _dev_ptr(image, "image"),
                                     _dev_ptr(sino_meas, "sino_meas"), float(relaxation),
                                     _dev_ptr(work, "work"), int(batch), _stream_handle(stream)))


def fp_sirt_prepare(handle, stream=None) -> None:
    _check(_lib.fp_sirt_prepare(handle, _stream_handle(stream)))


def fp_sirt_step_multi(jobs, stream=None) -> None:
    """jobs: sequence of (handle, image, sino_meas, work, relaxation), batch 1 each."""
    arr = (FpSirtJob * max(len(jobs), 1))()
    for k, (h, image, sino_meas, work, relax) in enumerate(jobs):
        arr[k] = FpSirtJob(h.value if isinstance(h, ctypes.c_void_p) else h,
                           _dev_ptr(image, "image").value, _dev_ptr(sino_meas, "sino_meas").value,
                           _dev_ptr(work, "work").value, float(relax))
    _check(_lib.fp_sirt_step_multi(arr, len(jobs), _stream_handle(stream)))


def fp_count_nonzero(handle, stream=None) -> int:
    out = ctypes.c_int64()
    _check(_lib.fp_count_nonzero(handle, ctypes.byref(out), _stream_handle(stream)))
    return int(out.value)


def fp_geometry_device_bytes(handle) -> int:
    return int(_lib.fp_geometry_device_bytes(handle))


def fp_sirt_scratch_bytes(handle, batch=1) -> int:
    return int(_lib.fp_sirt_scratch_bytes(handle, int(batch)))


def fp_geometry_quarter_turn(handle) -> bool:
    return bool(_lib.fp_geometry_quarter_turn(handle))


def fp_geometry_symmetry(handle) -> int:
    return int(_lib.fp_geometry_symmetry(handle))


# -- convenience wrapper --------------------------------------------------------

class Geometry:
    """Owns an ``fp_geometry`` and allocates outputs with torch.

    Images are ``[batch, ny, nx]`` (or ``[ny, nx]``), sinograms
    ``[batch, n_views, n_det]`` (or ``[n_views, n_det]``), float32 on the
    geometry's GPU.  ``beam`` is "flat" (fan beam, flat detector), "arc" (fan
    beam, arc detector) or "parallel"; ``det_pitch`` defaults to the width.
    """

    def __init__(self, nx, ny, pixel, dsc, dsd, angles, n_det, det_width, beam="flat",
                 det_pitch=None):
        self.nx, self.ny, self.n_det = int(nx), int(ny), int(n_det)
        self.angles = np.asarray(angles, dtype=np.float64)
        self.n_views = int(self.angles.size)
        self.pixel, self.dsc, self.dsd, self.det_width = float(pixel), float(dsc), float(dsd), float(det_width)
        self.det_pitch = float(det_width if det_pitch is None else det_pitch)
        self.beam = beam
        if beam == "flat" and det_pitch is None:
            self.handle = fp_geometry_create(nx, ny, pixel, dsc, dsd, self.angles, n_det, det_width)
        else:
            self.handle = fp_geometry_create_desc(BEAMS[beam], nx, ny, pixel, dsc, dsd, self.angles,
                                                  n_det, self.det_pitch, det_width)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            fp_geometry_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, t, shape, name):
        """Batch size of a [batch, *shape] or [*shape] tensor; anything else is
        rejected before it reaches the kernels."""
        if t.dim() not in (len(shape), len(shape) + 1) or tuple(t.shape[-len(shape):]) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)} or "
                             f"(batch, *{tuple(shape)})")
        return 1 if t.dim() == len(shape) else t.shape[0]

    def _output(self, out, like, b, shape, dtype, name):
        """The caller's output tensor, checked to hold exactly `b` results of
        `shape`, or a new one."""
        import torch
        full = shape if like.dim() == len(shape) else (b, *shape)
        if out is None:
            return torch.empty(full, dtype=dtype, device=like.device)
        if tuple(out.shape) != tuple(full) and not (b == 1 and tuple(out.shape) == tuple(shape)):
            raise ValueError(f"{name} has shape {tuple(out.shape)}, expected {tuple(full)}")
        return out

    def forward(self, image, out=None, stream=None):
        """A c for float32 (production kernels) or float64 (FP64 kernels)."""
        import torch
        b = self._batch(image, (self.ny, self.nx), "image")
        out = self._output(out, image, b, (self.n_views, self.n_det), image.dtype, "out")
        (fp_forward_f64 if image.dtype == torch.float64 else fp_forward)(self.handle, image, out, b,
                                                                          stream)
        return out

    def back(self, sino, out=None, stream=None):
        """A^T y for float32 (production kernels) or float64 (FP64 kernels)."""
        import torch
        b = self._batch(sino, (self.n_views, self.n_det), "sino")
        out = self._output(out, sino, b, (self.ny, self.nx), sino.dtype, "out")
        (fp_back_f64 if sino.dtype == torch.float64 else fp_back)(self.handle, sino, out, b, stream)
        return out

    def forward_reference(self, image, out=None, quad_points=0, stream=None):
        """The exact reference projection (FP64) of an image or a batch."""
        import torch
        b = self._batch(image, (self.ny, self.nx), "image")
        out = self._output(out, image, b, (self.n_views, self.n_det), torch.float64, "out")
        fp_forward_reference(self.handle, image, out, b, quad_points, stream)
        return out

    def back_reference(self, sino, out=None, quad_points=0, stream=None):
        """The adjoint of forward_reference (FP64)."""
        import torch
        b = self._batch(sino, (self.n_views, self.n_det), "sino")
        out = self._output(out, sino, b, (self.ny, self.nx), torch.float64, "out")
        fp_back_reference(self.handle, sino, out, b, quad_points, stream)
        return out

    def sirt_step(self, image, sino_meas, relaxation=1.0, work=None, stream=None):
        import torch
        b = self._batch(image, (self.ny, self.nx), "image")
        if self._batch(sino_meas, (self.n_views, self.n_det), "sino_meas") != b:
            raise ValueError("sino_meas and image hold different batch sizes")
        work = self._output(work, image, b, (self.n_views, self.n_det), torch.float32, "work")
        fp_sirt_step(self.handle, image, sino_meas, relaxation, work, b, stream)
        return image

    def count_nonzero(self, stream=None) -> int:
        return fp_count_nonzero(self.handle, stream)

    def device_bytes(self) -> int:
        return fp_geometry_device_bytes(self.handle)

    def sirt_scratch_bytes(self, batch=1) -> int:
        return fp_sirt_scratch_bytes(self.handle, batch)

    def quarter_turn(self) -> bool:
        """Whether FP32 projections run in the quarter-turn form."""
        return fp_geometry_quarter_turn(self.handle)

    def symmetry(self) -> int:
        """Order of the scan symmetry the FP32 projections use: 8 (quarter
        turns and the diagonal reflection: the back projection evaluates
        each entry for eight views, the forward for four), 4 (quarter turns)
        or 1."""
        return fp_geometry_symmetry(self.handle)
