"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the public header declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fanproj.h")
LIB = os.path.join(ROOT, "paper_1907_10526_amd", "libfanproj.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1907_10526_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"fp_geometry_create", "fp_forward", "fp_back", "fp_sirt_step"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_1907_10526_amd import fanproj
    assert sorted(fanproj.EXPORTED) == _declared()
    for n in fanproj.EXPORTED:
        assert callable(getattr(fanproj, n))


def _create(lib, **kw):
    args = dict(nx=64, ny=64, pixel=1.0, dsc=128.0, dsd=256.0, n_views=4, n_det=128, width=1.5)
    args.update(kw)
    ang = np.linspace(0, 1, max(args["n_views"], 1))
    out = ctypes.c_void_p()
    f = lib.fp_geometry_create
    f.restype = ctypes.c_int
    st = f(ctypes.c_int32(args["nx"]), ctypes.c_int32(args["ny"]), ctypes.c_double(args["pixel"]),
           ctypes.c_double(args["dsc"]), ctypes.c_double(args["dsd"]), ctypes.c_int32(args["n_views"]),
           ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_int32(args["n_det"]),
           ctypes.c_double(args["width"]), ctypes.byref(out))
    lib.fp_last_error.restype = ctypes.c_char_p
    return st, lib.fp_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(nx=0), ">= 1"), (dict(n_det=0), ">= 1"), (dict(n_views=0), ">= 1"),
    (dict(pixel=-1.0), "finite"), (dict(pixel=float("nan")), "finite"),
    (dict(width=0.0), "finite"), (dict(dsd=100.0), "exceed"),
    (dict(dsc=40.0, dsd=300.0), "outside the image"),
])
def test_invalid_geometry_rejected_without_device(lib, kw, needle):
    st, msg = _create(lib, **kw)
    assert st == 1, (st, msg)
    assert needle in msg


def test_null_arguments_rejected(lib):
    lib.fp_forward.restype = ctypes.c_int
    assert lib.fp_forward(None, None, None, ctypes.c_int32(1), None) == 1
    lib.fp_back.restype = ctypes.c_int
    assert lib.fp_back(None, None, None, ctypes.c_int32(1), None) == 1
    lib.fp_sirt_step.restype = ctypes.c_int
    assert lib.fp_sirt_step(None, None, None, ctypes.c_float(1.0), None, ctypes.c_int32(1), None) == 1
    lib.fp_geometry_device_bytes.restype = ctypes.c_size_t
    assert lib.fp_geometry_device_bytes(None) == 0
    lib.fp_geometry_destroy.restype = ctypes.c_int
    assert lib.fp_geometry_destroy(None) == 0
    lib.fp_last_error.restype = ctypes.c_char_p
    out = ctypes.c_int64()
    lib.fp_count_nonzero.restype = ctypes.c_int
    assert lib.fp_count_nonzero(None, ctypes.byref(out), None) == 1
    assert b"NULL" in lib.fp_last_error()


def _create_desc(lib, **kw):
    from paper_1907_10526_amd import fanproj
    args = dict(beam=0, nx=64, ny=64, pixel=1.0, dsc=128.0, dsd=256.0, n_views=4, n_det=128,
                pitch=1.5, width=1.5)
    args.update(kw)
    ang = np.linspace(0, 1, max(args["n_views"], 1))
    d = fanproj.FpGeometryDesc(args["beam"], args["nx"], args["ny"], args["pixel"], args["dsc"],
                               args["dsd"], args["n_views"],
                               ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), args["n_det"],
                               args["pitch"], args["width"])
    out = ctypes.c_void_p()
    f = lib.fp_geometry_create_desc
    f.restype = ctypes.c_int
    st = f(ctypes.byref(d), ctypes.byref(out))
    lib.fp_last_error.restype = ctypes.c_char_p
    return st, lib.fp_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(beam=7), "unknown beam"), (dict(pitch=0.0), "pitch"), (dict(pitch=float("inf")), "pitch"),
    (dict(beam=1, n_det=2000, pitch=0.5), "80 degrees"), (dict(beam=1, dsd=100.0), "exceed"),
    (dict(beam=2, nx=0), ">= 1"), (dict(beam=2, width=-1.0), "finite"),
])
def test_invalid_description_rejected_without_device(lib, kw, needle):
    st, msg = _create_desc(lib, **kw)
    assert st == 1, (st, msg)
    assert needle in msg


def test_parallel_description_ignores_distances(lib):
    # distances a fan geometry would reject pass validation for parallel
    # beams; on a host without a device the call then fails at the device
    st, msg = _create_desc(lib, beam=2, dsc=0.0, dsd=float("nan"))
    assert st != 1, msg


def test_null_description_rejected(lib):
    out = ctypes.c_void_p()
    lib.fp_geometry_create_desc.restype = ctypes.c_int
    assert lib.fp_geometry_create_desc(None, ctypes.byref(out)) == 1
