"""Differentiable 3D DRT and DJT: torch.autograd.Function wrappers of the HIP
transforms.

The DRT of planes is linear, R: R^{N^3} -> R^{K x N x N x (3N-2)}, so its
vector-Jacobian product is the backprojection R^T applied to the incoming
gradient (eqs. (16)-(17), Sec. 5: the reverse recursion). Nothing of the forward
is saved for the backward: no input, no stage buffer. The backward re-runs the
reverse recursion on the incoming gradient alone, which is the cheapest form of
recomputing stages instead of storing the log2(N) intermediates.

Two mutually adjoint Functions are defined so that higher derivatives work:
the backward of ``drt3d`` is ``drt3d_backproject`` and vice versa. The DJT of
lines (eq. (13), Sec. 4.1) gets the same pair, ``djt3d`` and
``djt3d_backproject``, over its reverse recursion (eq. (18)).

Volumes are float32 (int32 is accepted for the forward value but carries no
gradient). A leading batch dimension is accepted: a [B, N, N, N] input goes
through one batched launch sequence for the whole batch (forward and backward),
instead of B per-volume launch sequences.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api

__all__ = ["drt3d", "drt3d_backproject", "DRT3D", "DRT3DFunction", "DRT3DBackprojectFunction",
           "djt3d", "djt3d_backproject", "DJT3D", "DJT3DFunction", "DJT3DBackprojectFunction"]


def _check_mask(mask: int) -> int:
    mask = int(mask)
    if mask <= 0 or mask & ~api.DRT3D_ALL:
        raise ValueError("mask must be a nonzero 12-bit dodecant set, got %#x" % mask)
    return mask


class _Ops:
    """The single and batched calls and output shape of one transform."""

    def __init__(self, name, fwd, fwd_b, adj, adj_b, shape):
        self.name, self.fwd, self.fwd_b, self.adj, self.adj_b, self.shape = name, fwd, fwd_b, adj, adj_b, shape


_DRT = _Ops("DRT", api.drt3d_forward, api.drt3d_forward_batched, api.drt3d_adjoint, api.drt3d_adjoint_batched,
            api.drt3d_out_shape)
_DJT = _Ops("DJT", api.djt3d_forward, api.djt3d_forward_batched, api.djt3d_adjoint, api.djt3d_adjoint_batched,
            api.djt3d_out_shape)


def _forward_impl(vol: torch.Tensor, mask: int, ops: _Ops = _DRT) -> torch.Tensor:
    vol = vol.contiguous()
    if vol.dim() == 3:
        return ops.fwd(vol, mask)
    if vol.dim() != 4:
        raise ValueError("expected [N,N,N] or [B,N,N,N], got %s" % (tuple(vol.shape),))
    B, N = int(vol.shape[0]), int(vol.shape[1])
    out = torch.empty((B,) + ops.shape(N, mask), dtype=vol.dtype, device=vol.device)
    if B:
        ops.fwd_b([vol[b] for b in range(B)], mask, outs=[out[b] for b in range(B)])
    return out


def _adjoint_impl(proj: torch.Tensor, mask: int, ops: _Ops = _DRT) -> torch.Tensor:
    proj = proj.contiguous()
    rank = len(ops.shape(2, mask))
    if proj.dim() == rank:
        return ops.adj(proj, mask)
    if proj.dim() != rank + 1:
        raise ValueError("expected a %s projection set with or without a batch dimension, got %s"
                         % (ops.name, tuple(proj.shape)))
    B, N = int(proj.shape[0]), int(proj.shape[2])
    out = torch.empty((B, N, N, N), dtype=proj.dtype, device=proj.device)
    if B:
        ops.adj_b([proj[b] for b in range(B)], mask, outs=[out[b] for b in range(B)])
    return out


class DRT3DFunction(torch.autograd.Function):
    """y = R_K f; the gradient is R_K^T applied to dL/dy."""

    @staticmethod
    def forward(ctx, vol: torch.Tensor, mask: int) -> torch.Tensor:
        ctx.mask = mask
        return _forward_impl(vol, mask)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        if not ctx.needs_input_grad[0]:
            return None, None
        return DRT3DBackprojectFunction.apply(grad_out, ctx.mask), None


class DRT3DBackprojectFunction(torch.autograd.Function):
    """f = R_K^T p; the gradient is R_K applied to dL/df."""

    @staticmethod
    def forward(ctx, proj: torch.Tensor, mask: int) -> torch.Tensor:
        ctx.mask = mask
        return _adjoint_impl(proj, mask)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        if not ctx.needs_input_grad[0]:
            return None, None
        return DRT3DFunction.apply(grad_out, ctx.mask), None


def drt3d(vol: torch.Tensor, mask: int = api.DRT3D_ALL) -> torch.Tensor:
    """Differentiable DRT of planes over the dodecants of `mask`.

    vol: [N,N,N] or [B,N,N,N] on a HIP device. Returns [K,N,N,3N-2] or
    [B,K,N,N,3N-2], K = popcount(mask)."""
    return DRT3DFunction.apply(vol, _check_mask(mask))


def drt3d_backproject(proj: torch.Tensor, mask: int = api.DRT3D_ALL) -> torch.Tensor:
    """Differentiable backprojection (exact transpose of `drt3d`)."""
    return DRT3DBackprojectFunction.apply(proj, _check_mask(mask))


class DRT3D(torch.nn.Module):
    """Module form of `drt3d` with a fixed dodecant set."""

    def __init__(self, mask: int = api.DRT3D_ALL):
        super().__init__()
        self.mask = _check_mask(mask)

    def forward(self, vol: torch.Tensor) -> torch.Tensor:
        return drt3d(vol, self.mask)

    def extra_repr(self) -> str:
        return "mask=%#05x" % self.mask


class DJT3DFunction(torch.autograd.Function):
    """y = J_K f; the gradient is J_K^T applied to dL/dy."""

    @staticmethod
    def forward(ctx, vol: torch.Tensor, mask: int) -> torch.Tensor:
        ctx.mask = mask
        return _forward_impl(vol, mask, _DJT)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        if not ctx.needs_input_grad[0]:
            return None, None
        return DJT3DBackprojectFunction.apply(grad_out, ctx.mask), None


class DJT3DBackprojectFunction(torch.autograd.Function):
    """f = J_K^T p; the gradient is J_K applied to dL/df."""

    @staticmethod
    def forward(ctx, proj: torch.Tensor, mask: int) -> torch.Tensor:
        ctx.mask = mask
        return _adjoint_impl(proj, mask, _DJT)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        if not ctx.needs_input_grad[0]:
            return None, None
        return DJT3DFunction.apply(grad_out, ctx.mask), None


def djt3d(vol: torch.Tensor, mask: int = api.DRT3D_ALL) -> torch.Tensor:
    """Differentiable DJT of lines over the dodecants of `mask`.

    vol: [N,N,N] or [B,N,N,N] on a HIP device, N <= 256. Returns
    [K,N,N,2N-1,2N-1] or [B,K,N,N,2N-1,2N-1], K = popcount(mask)."""
    return DJT3DFunction.apply(vol, _check_mask(mask))


def djt3d_backproject(proj: torch.Tensor, mask: int = api.DRT3D_ALL) -> torch.Tensor:
    """Differentiable DJT backprojection (exact transpose of `djt3d`)."""
    return DJT3DBackprojectFunction.apply(proj, _check_mask(mask))


class DJT3D(torch.nn.Module):
    """Module form of `djt3d` with a fixed dodecant set."""

    def __init__(self, mask: int = api.DRT3D_ALL):
        super().__init__()
        self.mask = _check_mask(mask)

    def forward(self, vol: torch.Tensor) -> torch.Tensor:
        return djt3d(vol, self.mask)

    def extra_repr(self) -> str:
        return "mask=%#05x" % self.mask
