"""The CNSF projector as differentiable torch operators.

``project(image, geom)`` is ``A c`` and ``backproject(sino, geom)`` is
``A^T y``.  Each one's backward is the other's hand-written HIP kernel (the
pair is exactly adjoint: both evaluate the same entries of eq. (18)), so
gradients of any loss built on them cost one projection per use.  FP32
tensors run the production kernels; FP64 tensors run the FP64 instantiation
(for finite-difference checks).
"""
from __future__ import annotations

import torch

from .fanproj import Geometry

__all__ = ["project", "backproject", "Projector", "power_norm_sq"]


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image: torch.Tensor, geom: Geometry) -> torch.Tensor:
        ctx.geom = geom
        return geom.forward(image.contiguous())

    @staticmethod
    def backward(ctx, grad_sino: torch.Tensor):
        return ctx.geom.back(grad_sino.contiguous()), None


class _BackProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sino: torch.Tensor, geom: Geometry) -> torch.Tensor:
        ctx.geom = geom
        return geom.back(sino.contiguous())

    @staticmethod
    def backward(ctx, grad_image: torch.Tensor):
        return ctx.geom.forward(grad_image.contiguous()), None


def project(image: torch.Tensor, geom: Geometry) -> torch.Tensor:
    """Differentiable forward projection, image [B,ny,nx] or [ny,nx] -> sinogram."""
    return _Project.apply(image, geom)


def backproject(sino: torch.Tensor, geom: Geometry) -> torch.Tensor:
    """Differentiable back projection (the adjoint), sinogram -> image."""
    return _BackProject.apply(sino, geom)


class Projector(torch.nn.Module):
    """``nn.Module`` holding a geometry; ``module(image)`` is ``A image``."""

    def __init__(self, geom: Geometry):
        super().__init__()
        self.geom = geom

    def forward(self, image: torch.Tensor) -> torch.Tensor:
        return project(image, self.geom)

    def adjoint(self, sino: torch.Tensor) -> torch.Tensor:
        return backproject(sino, self.geom)


@torch.no_grad()
def power_norm_sq(geom: Geometry, iters: int = 20, seed: int = 0,
                  device="cuda", dtype=torch.float32) -> float:
    """Estimate ||A||_2^2 (largest eigenvalue of A^T A) by power iteration."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.rand((geom.ny, geom.nx), generator=g, dtype=dtype).to(device)
    x /= x.norm()
    lam = 0.0
    for _ in range(iters):
        y = geom.back(geom.forward(x))
        lam = float((x * y).sum())
        x = y / y.norm()
    return lam
