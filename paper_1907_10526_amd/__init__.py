"""MI355X-native CNSF fan-beam forward and back projection (arXiv 1907.10526).

The projector itself is ``libfanproj.so`` (HIP kernels for gfx950 behind a C
ABI declared in ``include/fanproj.h``); :mod:`.fanproj` binds it.  The binding
is imported lazily so that the input generators can be used without a GPU.
"""
from . import phantoms, workloads  # noqa: F401  (no GPU or native code needed)

__all__ = ["phantoms", "workloads"]
