"""PyTorch autograd wrappers around the hand-written HIP adjoints.

The paper's askadam relies on automatic differentiation of the forward model
(§2.2.1); here every model has a hand-written vector-Jacobian product and the
TV term (§2.4, Eq. 5) its subgradient, both exposed through the C ABI and
wrapped as ``torch.autograd.Function`` so that user losses written in torch
differentiate through them.  Tensors must be float32, contiguous and on the
GPU; parameters are [P, n] (compacted voxels), signals [M_eff, n].
"""
from __future__ import annotations

import torch

from . import lib as _load


class ForwardModel(torch.autograd.Function):
    """s = f(theta) with backward dtheta = J(theta)^T ds (gc_model_forward / gc_model_vjp)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, model) -> torch.Tensor:
        g = _load()
        theta = theta.contiguous()
        ctx.model = model
        ctx.save_for_backward(theta)
        return g.gc_model_forward(model, theta)

    @staticmethod
    def backward(ctx, ds: torch.Tensor):
        g = _load()
        (theta,) = ctx.saved_tensors
        return g.gc_model_vjp(ctx.model, theta, ds.contiguous()), None


class TotalVariation(torch.autograd.Function):
    """R(u) = sum over masked forward-neighbour pairs |u_b - u_a| of a grid map
    u [nz, ny, nx] (gc_tv); backward multiplies the subgradient (sign(0) = 0)."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, mask, tv_dim: int = 3) -> torch.Tensor:
        g = _load()
        R, dR = g.gc_tv(u.contiguous(), mask, tv_dim=tv_dim, scale=1.0, grad=True)
        ctx.save_for_backward(dR)
        return torch.tensor(R, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, gR: torch.Tensor):
        (dR,) = ctx.saved_tensors
        return dR * gR.to(dR.dtype), None, None


class SenseOperator(torch.autograd.Function):
    """k = M_e F2(C_c I_e) of the reconstruction (paper §2.6.4, Eq. 7) for a
    complex64 image [E, Ny, Nz] (gc_sense_forward); backward applies the
    adjoint sum_c conj(C_c) F2^H(M_e dk) (gc_sense_adjoint), which for torch's
    complex gradients (dL/dRe + i dL/dIm) is the vector-Jacobian product."""

    @staticmethod
    def forward(ctx, image: torch.Tensor, coils: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
        g = _load()
        ctx.save_for_backward(coils, mask)
        return g.gc_sense_forward(image.contiguous(), coils, mask)

    @staticmethod
    def backward(ctx, dk: torch.Tensor):
        g = _load()
        coils, mask = ctx.saved_tensors
        return g.gc_sense_adjoint(dk.contiguous(), coils, mask), None, None


def forward_model(theta: torch.Tensor, model) -> torch.Tensor:
    return ForwardModel.apply(theta, model)


def total_variation(u: torch.Tensor, mask=None, tv_dim: int = 3) -> torch.Tensor:
    return TotalVariation.apply(u, mask, tv_dim)


def sense_operator(image: torch.Tensor, coils: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    return SenseOperator.apply(image, coils, mask)
