"""Torch-facing binding of the 2D kernel-sum representation (the paper's Section 3).

An RGB image is represented by K weighted isotropic kernels,
f_c(x) = sum over |x - mu_k| < D of A_kc exp(-|x - mu_k|^2 / sigma_k^2), with no
compositing. Binning, rendering and gradients run in the library's HIP kernels
(``isogs_field2d_bin`` / ``_fwd`` / ``_bwd`` of include/isogs.h); this module allocates
buffers and marshals arguments.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _abi as A
from .rasterizer import Footprints, TileBins, _alloc_bins, _p, _stream

_F32 = torch.float32


def _field(mu, sigma, amp) -> A.Field2D:
    f = A.Field2D()
    f.mu, f.sigma, f.amp = _p(mu), _p(sigma), _p(amp)
    f.K = int(sigma.shape[0])
    return f


def _check_params(mu, sigma, amp):
    K = int(sigma.shape[0])
    for name, x, shape in (("mu", mu, (2, K)), ("sigma", sigma, (K,)), ("amp", amp, (3, K))):
        if tuple(x.shape) != shape or x.dtype != _F32 or not x.is_contiguous() or not x.is_cuda:
            raise ValueError(f"{name}: need a contiguous CUDA float32 tensor of shape {shape}")


class Field2DRenderer:
    """Bins, renders and differentiates a 2D kernel-sum signal on a fixed image size and
    support radius, keeping the workspaces between calls. Every particle's support disk
    meets at most (ceil(2D/16) + 1)^2 tiles, so the entry capacity is sized from that
    bound (plus a margin of one tile per axis) and binning cannot overflow; an explicit
    smaller `capacity` is grown on demand (one host synchronisation)."""

    def __init__(self, width, height, support, device="cuda", headroom=1.25):
        self.width, self.height, self.support = int(width), int(height), float(support)
        self.device = torch.device(device)
        self.headroom = headroom
        self.capacity = 0
        self.tiles = ((self.width + 15) // 16) * ((self.height + 15) // 16)
        self._ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self._wsb = torch.empty(0, dtype=torch.uint8, device=self.device)

    @staticmethod
    def _grow(buf, nbytes):
        return buf if buf.numel() >= nbytes else torch.empty(int(nbytes), dtype=torch.uint8, device=buf.device)

    def tiles_bound(self) -> int:
        return (math.ceil(2.0 * self.support / 16.0) + 2) ** 2

    def bin(self, mu, sigma, amp, check=True, capacity=None):
        """Footprints and tile lists of the particles. With `check`, reads the device status
        (one synchronisation) and grows the capacity on overflow; without it nothing
        waits (safe at the default capacity, which no binning can exceed)."""
        _check_params(mu, sigma, amp)
        K = int(sigma.shape[0])
        fp = Footprints.empty(K, self.device)
        f = _field(mu, sigma, amp)
        if capacity is None:
            self.capacity = max(self.capacity, K * self.tiles_bound())
            cap = self.capacity
        else:
            cap = int(capacity)
        for _ in range(2):
            bins = _alloc_bins(cap, K, self.tiles, self.device)
            ab = bins.abi()
            need = ctypes.c_size_t(0)
            args = (ctypes.byref(f), self.width, self.height, self.support, ctypes.byref(fp.abi()), ctypes.byref(ab))
            A.check(A.lib().isogs_field2d_bin(*args, None, ctypes.byref(need), _stream()))
            self._ws = self._grow(self._ws, need.value)
            have = ctypes.c_size_t(self._ws.numel())
            A.check(A.lib().isogs_field2d_bin(*args, _p(self._ws), ctypes.byref(have), _stream()))
            if not check:
                return fp, bins
            st = int(bins.status.item())
            if st == A.ISOGS_OK:
                return fp, bins
            if st != A.ISOGS_ERR_CAPACITY:
                raise A.IsoGSError(st, "isogs_field2d_bin failed on the device")
            cap = int(bins.n_entries() * self.headroom) + 4096
            self.capacity = max(self.capacity, cap)
        raise A.IsoGSError(A.ISOGS_ERR_CAPACITY, "field2d capacity still too small after growing")

    def render(self, fp: Footprints, bins: TileBins, K: int, out=None):
        """The image [3, H, W]."""
        image = torch.empty((3, self.height, self.width), dtype=_F32, device=self.device) if out is None else out
        A.check(A.lib().isogs_field2d_fwd(ctypes.byref(fp.abi()), int(K), ctypes.byref(bins.abi()), self.width,
                                          self.height, self.support, _p(image), _stream()))
        return image

    def grads(self, fp: Footprints, bins: TileBins, K: int, dL_dimage):
        """(dL/dmu [2, K], dL/dsigma [K], dL/dA [3, K]) for dL/dimage [3, H, W]."""
        gmu = torch.empty((2, K), dtype=_F32, device=self.device)
        gsig = torch.empty(K, dtype=_F32, device=self.device)
        gamp = torch.empty((3, K), dtype=_F32, device=self.device)
        g = _field(gmu, gsig, gamp)
        dl = dL_dimage.contiguous()
        need = ctypes.c_size_t(0)
        args = (ctypes.byref(fp.abi()), int(K), ctypes.byref(bins.abi()), self.width, self.height, self.support,
                _p(dl), ctypes.byref(g))
        A.check(A.lib().isogs_field2d_bwd(*args, None, ctypes.byref(need), _stream()))
        self._wsb = self._grow(self._wsb, max(need.value, 1))
        have = ctypes.c_size_t(self._wsb.numel())
        A.check(A.lib().isogs_field2d_bwd(*args, _p(self._wsb), ctypes.byref(have), _stream()))
        return gmu, gsig, gamp


def _field_aniso(mu, theta, scale, amp) -> A.Field2DAniso:
    f = A.Field2DAniso()
    f.mu, f.theta, f.scale, f.amp = _p(mu), _p(theta), _p(scale), _p(amp)
    f.K = int(theta.shape[0])
    return f


class Field2DAnisoRenderer(Field2DRenderer):
    """The same renderer for anisotropic kernels (isogs_field2d_aniso_*): particles with
    centre mu [2, K], rotation angle theta [K], scales [2, K] and amplitude [3, K]. bin()
    returns (footprints, conic_c, bins)."""

    def bin(self, mu, theta, scale, amp, check=True, capacity=None):
        K = int(theta.shape[0])
        for name, x, shape in (("mu", mu, (2, K)), ("theta", theta, (K,)), ("scale", scale, (2, K)),
                               ("amp", amp, (3, K))):
            if tuple(x.shape) != shape or x.dtype != _F32 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError(f"{name}: need a contiguous CUDA float32 tensor of shape {shape}")
        fp = Footprints.empty(K, self.device)
        conic_c = torch.empty(max(K, 1), dtype=_F32, device=self.device)
        f = _field_aniso(mu, theta, scale, amp)
        if capacity is None:
            self.capacity = max(self.capacity, K * self.tiles_bound())
            cap = self.capacity
        else:
            cap = int(capacity)
        for _ in range(2):
            bins = _alloc_bins(cap, K, self.tiles, self.device)
            ab = bins.abi()
            need = ctypes.c_size_t(0)
            args = (ctypes.byref(f), self.width, self.height, self.support, ctypes.byref(fp.abi()), _p(conic_c),
                    ctypes.byref(ab))
            A.check(A.lib().isogs_field2d_aniso_bin(*args, None, ctypes.byref(need), _stream()))
            self._ws = self._grow(self._ws, need.value)
            have = ctypes.c_size_t(self._ws.numel())
            A.check(A.lib().isogs_field2d_aniso_bin(*args, _p(self._ws), ctypes.byref(have), _stream()))
            if not check:
                return fp, conic_c, bins
            st = int(bins.status.item())
            if st == A.ISOGS_OK:
                return fp, conic_c, bins
            if st != A.ISOGS_ERR_CAPACITY:
                raise A.IsoGSError(st, "isogs_field2d_aniso_bin failed on the device")
            cap = int(bins.n_entries() * self.headroom) + 4096
            self.capacity = max(self.capacity, cap)
        raise A.IsoGSError(A.ISOGS_ERR_CAPACITY, "field2d capacity still too small after growing")

    def render(self, fp: Footprints, conic_c, bins: TileBins, K: int, out=None):
        image = torch.empty((3, self.height, self.width), dtype=_F32, device=self.device) if out is None else out
        A.check(A.lib().isogs_field2d_aniso_fwd(ctypes.byref(fp.abi()), _p(conic_c), int(K), ctypes.byref(bins.abi()),
                                                self.width, self.height, self.support, _p(image), _stream()))
        return image

    def grads(self, mu, theta, scale, amp, fp: Footprints, conic_c, bins: TileBins, dL_dimage):
        """(dL/dmu [2, K], dL/dtheta [K], dL/dscale [2, K], dL/dA [3, K])."""
        K = int(theta.shape[0])
        out = (torch.empty((2, K), dtype=_F32, device=self.device), torch.empty(K, dtype=_F32, device=self.device),
               torch.empty((2, K), dtype=_F32, device=self.device), torch.empty((3, K), dtype=_F32, device=self.device))
        f, g = _field_aniso(mu, theta, scale, amp), _field_aniso(*out)
        need = ctypes.c_size_t(0)
        args = (ctypes.byref(f), ctypes.byref(fp.abi()), _p(conic_c), ctypes.byref(bins.abi()), self.width,
                self.height, self.support, _p(dL_dimage.contiguous()), ctypes.byref(g))
        A.check(A.lib().isogs_field2d_aniso_bwd(*args, None, ctypes.byref(need), _stream()))
        self._wsb = self._grow(self._wsb, max(need.value, 1))
        have = ctypes.c_size_t(self._wsb.numel())
        A.check(A.lib().isogs_field2d_aniso_bwd(*args, _p(self._wsb), ctypes.byref(have), _stream()))
        return out


class Field2DAnisoRender(torch.autograd.Function):
    """Differentiable image of an anisotropic 2D kernel sum: forward(mu, theta, scale, amp,
    renderer) -> [3, H, W]; gradients flow to all four parameter tensors."""

    @staticmethod
    def forward(ctx, mu, theta, scale, amp, renderer):
        mu, theta, scale, amp = mu.contiguous(), theta.contiguous(), scale.contiguous(), amp.contiguous()
        fp, conic_c, bins = renderer.bin(mu, theta, scale, amp, check=False)
        image = renderer.render(fp, conic_c, bins, int(theta.shape[0]))
        ctx.renderer, ctx.fp, ctx.conic_c, ctx.bins = renderer, fp, conic_c, bins
        ctx.save_for_backward(mu, theta, scale, amp)
        return image

    @staticmethod
    def backward(ctx, grad_out):
        mu, theta, scale, amp = ctx.saved_tensors
        g = ctx.renderer.grads(mu, theta, scale, amp, ctx.fp, ctx.conic_c, ctx.bins, grad_out)
        return (*g, None)


def _alloc_params(cap, device):
    return (torch.empty((2, cap), dtype=_F32, device=device), torch.empty(cap, dtype=_F32, device=device),
            torch.empty((3, cap), dtype=_F32, device=device))


def tree_init(target, K, root=64, min_side=2, tau=1e-3):
    """Quadtree initialisation (isogs_field2d_tree_init) of particles for `target` [3, H, W]:
    returns (mu [2, n], sigma [n], amp [3, n]), n <= K (one host synchronisation for n)."""
    target = target.contiguous()
    if target.dim() != 3 or target.shape[0] != 3 or target.dtype != _F32 or not target.is_cuda:
        raise ValueError("target: need a CUDA float32 tensor [3, H, W]")
    H, W = int(target.shape[1]), int(target.shape[2])
    out = _alloc_params(int(K), target.device)
    count = torch.zeros(1, dtype=torch.int32, device=target.device)
    fo = _field(*out)
    need = ctypes.c_size_t(0)
    args = (_p(target), H, W, int(root), int(min_side), float(tau), int(K), ctypes.byref(fo), _p(count))
    A.check(A.lib().isogs_field2d_tree_init(*args, None, ctypes.byref(need), _stream()))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=target.device)
    have = ctypes.c_size_t(ws.numel())
    A.check(A.lib().isogs_field2d_tree_init(*args, _p(ws), ctypes.byref(have), _stream()))
    n = int(count.item())
    return out[0][:, :n].contiguous(), out[1][:n].contiguous(), out[2][:, :n].contiguous()


def _edit(fn, mu, sigma, amp, thr, factor):
    _check_params(mu, sigma, amp)
    K = int(sigma.shape[0])
    cap = max(1, factor * K)
    out = _alloc_params(cap, mu.device)
    count = torch.zeros(1, dtype=torch.int32, device=mu.device)
    fi, fo = _field(mu, sigma, amp), _field(*out)
    need = ctypes.c_size_t(0)
    A.check(fn(ctypes.byref(fi), float(thr), ctypes.byref(fo), _p(count), None, ctypes.byref(need), _stream()))
    ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=mu.device)
    have = ctypes.c_size_t(ws.numel())
    A.check(fn(ctypes.byref(fi), float(thr), ctypes.byref(fo), _p(count), _p(ws), ctypes.byref(have), _stream()))
    n = int(count.item())
    return out[0][:, :n].contiguous(), out[1][:n].contiguous(), out[2][:, :n].contiguous()


def prune(mu, sigma, amp, amp_min):
    """Drops particles whose max_c |A_kc| < amp_min (isogs_field2d_prune), keeping order."""
    return _edit(A.lib().isogs_field2d_prune, mu, sigma, amp, amp_min, 1)


def split(mu, sigma, amp, sigma_max):
    """Replaces every particle with sigma > sigma_max by four of half its scale
    (isogs_field2d_split), in place in the order."""
    return _edit(A.lib().isogs_field2d_split, mu, sigma, amp, sigma_max, 4)


def merge(mu, sigma, amp, width, height, cell, sigma_max):
    """Merges the particles with sigma <= sigma_max whose centres share a cell of edge `cell`
    (isogs_field2d_merge): each group of two or more becomes one particle keeping the
    kernels' mass per channel, at the place of its first member; the inverse of split."""
    _check_params(mu, sigma, amp)
    K = int(sigma.shape[0])
    out = _alloc_params(max(1, K), mu.device)
    count = torch.zeros(1, dtype=torch.int32, device=mu.device)
    fi, fo = _field(mu, sigma, amp), _field(*out)
    args = (ctypes.byref(fi), int(width), int(height), float(cell), float(sigma_max), ctypes.byref(fo), _p(count))
    need = ctypes.c_size_t(0)
    A.check(A.lib().isogs_field2d_merge(*args, None, ctypes.byref(need), _stream()))
    ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=mu.device)
    have = ctypes.c_size_t(ws.numel())
    A.check(A.lib().isogs_field2d_merge(*args, _p(ws), ctypes.byref(have), _stream()))
    n = int(count.item())
    return out[0][:, :n].contiguous(), out[1][:n].contiguous(), out[2][:, :n].contiguous()


def octree_init(points, colors, lo, root_side, roots, levels, tau, K, opacity=0.5, sh_degree=0):
    """Octree initialisation of 3D particles (isogs_octree_init) from a coloured point cloud
    (points, colors: CUDA float32 [3, P]): returns a GaussianScene of at most K particles
    (one host synchronisation for the count) and the number of leaves."""
    from .rasterizer import GaussianScene
    points, colors = points.contiguous(), colors.contiguous()
    for name, x in (("points", points), ("colors", colors)):
        if x.dim() != 2 or x.shape[0] != 3 or x.dtype != _F32 or not x.is_cuda:
            raise ValueError(f"{name}: need a CUDA float32 tensor [3, P]")
    dev = points.device
    Kc = (int(sh_degree) + 1) ** 2
    out = GaussianScene(torch.empty((3, K), dtype=_F32, device=dev), torch.empty(K, dtype=_F32, device=dev),
                        torch.empty(K, dtype=_F32, device=dev), torch.empty((3 * Kc, K), dtype=_F32, device=dev),
                        int(sh_degree))
    g = A.OctreeGrid()
    g.lo[:] = [float(x) for x in lo]
    g.root_side = float(root_side)
    g.roots[:] = [int(x) for x in roots]
    g.levels = int(levels)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    so = out.abi()
    args = (_p(points), _p(colors), int(points.shape[1]), ctypes.byref(g), float(tau), int(K), float(opacity),
            ctypes.byref(so), _p(count))
    need = ctypes.c_size_t(0)
    A.check(A.lib().isogs_octree_init(*args, None, ctypes.byref(need), _stream()))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    have = ctypes.c_size_t(ws.numel())
    A.check(A.lib().isogs_octree_init(*args, _p(ws), ctypes.byref(have), _stream()))
    total = int(count.item())
    n = min(total, int(K))
    scene = GaussianScene(out.pos[:, :n].contiguous(), out.scale[:n].contiguous(), out.opacity[:n].contiguous(),
                          out.color[:, :n].contiguous(), int(sh_degree))
    return scene, total


class Field2DRender(torch.autograd.Function):
    """Differentiable image of a 2D kernel-sum signal: forward(mu, sigma, amp, renderer)
    -> [3, H, W]; gradients flow to mu [2, K], sigma [K] and amp [3, K]. Nothing waits on
    the host: the renderer's capacity bound rules out an overflow."""

    @staticmethod
    def forward(ctx, mu, sigma, amp, renderer):
        mu, sigma, amp = mu.contiguous(), sigma.contiguous(), amp.contiguous()
        fp, bins = renderer.bin(mu, sigma, amp, check=False)
        image = renderer.render(fp, bins, int(sigma.shape[0]))
        ctx.renderer, ctx.fp, ctx.bins, ctx.K = renderer, fp, bins, int(sigma.shape[0])
        return image

    @staticmethod
    def backward(ctx, grad_out):
        gmu, gsig, gamp = ctx.renderer.grads(ctx.fp, ctx.bins, ctx.K, grad_out)
        return gmu, gsig, gamp, None
