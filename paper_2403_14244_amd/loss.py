"""The paper's loss (Section 3): (1 - lambda) L1 + lambda (1 - SSIM), lambda = 0.2.

Both terms and their gradients run in the library's HIP kernels (``isogs_l1_fwd`` /
``_bwd`` and ``isogs_ssim_fwd`` / ``_bwd`` of include/isogs.h; SSIM: 11 x 11 Gaussian
window, sigma 1.5, zero outside the image, C1 = 0.01^2, C2 = 0.03^2). This module
marshals arguments only.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi as A
from .rasterizer import _p, _stream

LAMBDA = 0.2


def _planes(x):
    """[..., H, W] -> (planes, H, W) of a contiguous float32 CUDA tensor."""
    if x.dim() < 2 or x.dtype != torch.float32 or not x.is_cuda:
        raise ValueError("need a CUDA float32 tensor of shape [..., H, W]")
    H, W = int(x.shape[-2]), int(x.shape[-1])
    return max(1, x.numel() // (H * W)), H, W


class SSIM(torch.autograd.Function):
    """Mean SSIM of `image` against the constant `target` (same shape [..., H, W], every
    leading index a separate plane); differentiable in `image`."""

    @staticmethod
    def forward(ctx, image, target):
        image, target = image.contiguous(), target.contiguous()
        if image.shape != target.shape:
            raise ValueError("image and target must have the same shape")
        C, H, W = _planes(image)
        need = ctypes.c_size_t(0)
        A.check(A.lib().isogs_ssim_fwd(None, None, C, H, W, None, None, ctypes.byref(need), _stream()))
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=image.device)
        out = torch.empty(1, dtype=torch.float32, device=image.device)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_ssim_fwd(_p(image), _p(target), C, H, W, _p(out), _p(ws), ctypes.byref(have),
                                       _stream()))
        ctx.save_for_backward(image, target)
        ctx.ws, ctx.dims = ws, (C, H, W)
        return out[0]

    @staticmethod
    def backward(ctx, grad_out):
        image, target = ctx.saved_tensors
        C, H, W = ctx.dims
        g = grad_out.reshape(1).to(torch.float32).contiguous()
        dimg = torch.empty_like(image)
        A.check(A.lib().isogs_ssim_bwd(_p(image), _p(target), C, H, W, _p(g), _p(ctx.ws), ctx.ws.numel(), _p(dimg),
                                       _stream()))
        return dimg, None


class L1(torch.autograd.Function):
    """mean |image - target| (target constant), two kernels forward, one backward."""

    @staticmethod
    def forward(ctx, image, target):
        image, target = image.contiguous(), target.contiguous()
        if image.shape != target.shape or image.dtype != torch.float32 or not image.is_cuda:
            raise ValueError("image and target: CUDA float32 tensors of one shape")
        n = image.numel()
        need = ctypes.c_size_t(0)
        A.check(A.lib().isogs_l1_fwd(None, None, n, None, None, ctypes.byref(need), _stream()))
        ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=image.device)
        out = torch.empty(1, dtype=torch.float32, device=image.device)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_l1_fwd(_p(image), _p(target), n, _p(out), _p(ws), ctypes.byref(have), _stream()))
        ctx.save_for_backward(image, target)
        return out[0]

    @staticmethod
    def backward(ctx, grad_out):
        image, target = ctx.saved_tensors
        g = grad_out.reshape(1).to(torch.float32).contiguous()
        dimg = torch.empty_like(image)
        A.check(A.lib().isogs_l1_bwd(_p(image), _p(target), image.numel(), _p(g), _p(dimg), _stream()))
        return dimg, None


class L1SSIMLoss(torch.autograd.Function):
    """(1 - lam) mean|image - target| + lam (1 - SSIM(image, target)) in the library: one
    forward call (both terms and their combination), one fused gradient kernel."""

    @staticmethod
    def forward(ctx, image, target, lam):
        image, target = image.contiguous(), target.contiguous()
        if image.shape != target.shape:
            raise ValueError("image and target must have the same shape")
        C, H, W = _planes(image)
        need = ctypes.c_size_t(0)
        A.check(A.lib().isogs_loss_fwd(None, None, C, H, W, float(lam), None, None, ctypes.byref(need), _stream()))
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=image.device)
        out = torch.empty(2, dtype=torch.float32, device=image.device)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_loss_fwd(_p(image), _p(target), C, H, W, float(lam), _p(out), _p(ws),
                                       ctypes.byref(have), _stream()))
        ctx.save_for_backward(image, target)
        ctx.ws, ctx.dims, ctx.lam = ws, (C, H, W), float(lam)
        return out[0]

    @staticmethod
    def backward(ctx, grad_out):
        image, target = ctx.saved_tensors
        C, H, W = ctx.dims
        g = grad_out.reshape(1).to(torch.float32).contiguous()
        dimg = torch.empty_like(image)
        A.check(A.lib().isogs_loss_bwd(_p(image), _p(target), C, H, W, ctx.lam, _p(g), _p(ctx.ws), ctx.ws.numel(),
                                       _p(dimg), _stream()))
        return dimg, None, None


def ssim(image, target):
    return SSIM.apply(image, target)


def l1_loss(image, target):
    """mean |image - target|, differentiable in `image`."""
    return L1.apply(image, target)


def l1_ssim_loss(image, target, lam=LAMBDA):
    """(1 - lam) mean|image - target| + lam (1 - SSIM(image, target)), value and gradient
    formed in the library (isogs_loss_fwd / _bwd)."""
    return L1SSIMLoss.apply(image, target, lam)
