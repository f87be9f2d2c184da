"""Torch-facing binding of the anisotropic variant (eq. 5-7): particles with a rotation and
three scales, conic footprints, the same bins, sort and compositing walks.

Argument marshalling only: every step runs in the library's HIP kernels
(isogs_aniso_project, isogs_bin_sort, isogs_aniso_render_fwd, isogs_aniso_render_bwd).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi as A
from .rasterizer import Footprints, Rasterizer, TileBins, _p, _stream, sh_count

_F32 = torch.float32


@dataclass
class AnisoGaussianScene:
    """pos [3, N], rot [4, N] quaternions (w, x, y, z), scale [3, N] (linear per axis),
    opacity [N] (activated), color [3K, N]; device FP32."""
    pos: torch.Tensor
    rot: torch.Tensor
    scale: torch.Tensor
    opacity: torch.Tensor
    color: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    @staticmethod
    def from_host(scene, device="cuda") -> "AnisoGaussianScene":
        """From any object with numpy pos/rot/scale/opacity/color/sh_degree (scenegen.AnisoScene)."""
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return AnisoGaussianScene(t(scene.pos), t(scene.rot), t(scene.scale), t(scene.opacity), t(scene.color),
                                  int(scene.sh_degree))

    def validate(self):
        n = self.n
        K = sh_count(self.sh_degree)
        for name, x, shape in (("pos", self.pos, (3, n)), ("rot", self.rot, (4, n)), ("scale", self.scale, (3, n)),
                               ("opacity", self.opacity, (n,)), ("color", self.color, (3 * K, n))):
            if tuple(x.shape) != shape or x.dtype != _F32 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError(f"scene.{name}: need a contiguous CUDA float32 tensor of shape {shape}")

    def abi(self) -> A.AnisoScene:
        s = A.AnisoScene()
        s.pos, s.rot, s.scale = _p(self.pos), _p(self.rot), _p(self.scale)
        s.opacity, s.color = _p(self.opacity), _p(self.color)
        s.n = self.n
        s.sh_degree = self.sh_degree
        return s

    def empty_like(self) -> "AnisoGaussianScene":
        return AnisoGaussianScene(*(torch.empty_like(x) for x in (self.pos, self.rot, self.scale, self.opacity,
                                                                  self.color)), self.sh_degree)


@dataclass
class AnisoFootprints:
    """Output of the anisotropic projection: the record layout of Footprints (with A in
    place of 1/s^2: {u, v, A, o, r, g, b, radius}) plus the conic's {B, C} [N, 2]."""
    fp: Footprints
    conic: torch.Tensor

    @property
    def record(self):
        return self.fp.record

    @property
    def depth(self):
        return self.fp.depth

    @property
    def tile_count(self):
        return self.fp.tile_count

    def abi(self) -> A.Projected:
        """What binning reads (isogs_bin_sort takes the isotropic record layout)."""
        return self.fp.abi()

    def aniso_abi(self) -> A.AnisoProjected:
        p = A.AnisoProjected()
        p.fp = self.fp.abi()
        p.conic = _p(self.conic)
        return p

    @staticmethod
    def empty(n, device="cuda") -> "AnisoFootprints":
        return AnisoFootprints(Footprints.empty(n, device), torch.empty((n, 2), dtype=_F32, device=device))


class AnisoRasterizer(Rasterizer):
    """Rasterizer of anisotropic particles: project -> bin_sort (shared) -> longest-first
    compositing -> backward, through the anisotropic calls of the C ABI."""

    def __init__(self, device="cuda", headroom=1.25):
        super().__init__(device, headroom)
        self.ordered_fwd = True   # the anisotropic family has the longest-first walk only

    def project(self, scenes, cams) -> AnisoFootprints:
        n_total = sum(s.n for s in scenes)
        af = AnisoFootprints.empty(n_total, self.device)
        sc = (A.AnisoScene * len(scenes))(*[s.abi() for s in scenes])
        A.check(A.lib().isogs_aniso_project(sc, A.camera_array(cams), len(cams), ctypes.byref(af.aniso_abi()),
                                            _stream()))
        return af

    def render_fwd(self, *a, **k):
        raise NotImplementedError("the anisotropic family composites longest list first: use render_fwd_ordered")

    def render_fwd_ordered(self, af: AnisoFootprints, n_per_view, bins: TileBins, cams, bg=(0.0, 0.0, 0.0),
                           out=None, ckpt=None, wide=False, last=True):
        """`last=False`: no n_last (None), for a forward that no backward pass follows."""
        pix = sum(int(c.width) * int(c.height) for c in cams)
        if out is None:
            out = (torch.empty(3 * pix, dtype=_F32, device=self.device),
                   torch.empty(pix, dtype=_F32, device=self.device),
                   torch.empty(pix, dtype=torch.int32, device=self.device) if last else None)
        image, T, n_last = out
        bgc = (ctypes.c_float * 3)(*[float(b) for b in bg])
        args = (ctypes.byref(af.aniso_abi()), A.int_array(n_per_view), ctypes.byref(bins.abi()),
                A.camera_array(cams), len(cams), bgc, _p(image), _p(T), _p(n_last), _p(ckpt),
                A.ISOGS_FWD_WIDE if wide else 0)
        need = ctypes.c_size_t(0)
        A.check(A.lib().isogs_aniso_render_fwd(*args, None, ctypes.byref(need), _stream()))
        ws = self._workspace_q(need.value)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_aniso_render_fwd(*args, _p(ws), ctypes.byref(have), _stream()))
        return image, T, n_last

    def render_bwd(self, scenes, cams, af: AnisoFootprints, bins: TileBins, bg, dL_dimage, T_final, n_last,
                   grads=None, image=None, ckpt=None):
        """One AnisoGaussianScene of gradients per distinct scene (by pos pointer), in order of
        first appearance; views of one scene are summed in view order."""
        if grads is None:
            uniq = {}
            for s in scenes:
                if s.pos.data_ptr() not in uniq:
                    uniq[s.pos.data_ptr()] = s.empty_like()
            grads = [uniq[s.pos.data_ptr()] for s in scenes]
        sc = (A.AnisoScene * len(scenes))(*[s.abi() for s in scenes])
        gs = (A.AnisoScene * len(scenes))(*[g.abi() for g in grads])
        bgc = (ctypes.c_float * 3)(*[float(b) for b in bg])
        args = (sc, A.camera_array(cams), len(cams), ctypes.byref(af.aniso_abi()), ctypes.byref(bins.abi()), bgc,
                _p(image), _p(dL_dimage.contiguous()), _p(T_final), _p(n_last), _p(ckpt), gs)
        need = ctypes.c_size_t(0)
        A.check(A.lib().isogs_aniso_render_bwd(*args, None, ctypes.byref(need), _stream()))
        ws = self._workspace(need.value)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_aniso_render_bwd(*args, _p(ws), ctypes.byref(have), _stream()))
        out, seen = [], set()
        for g in grads:
            if g.pos.data_ptr() not in seen:
                seen.add(g.pos.data_ptr())
                out.append(g)
        return out


class AnisoGSRender(torch.autograd.Function):
    """Differentiable render of one anisotropic scene from V cameras of equal size.

    forward(pos, rot, scale, opacity, color, sh_degree, cams, bg, rasterizer) -> [V, 3, H, W];
    gradients flow to all five parameter tensors."""

    @staticmethod
    def forward(ctx, pos, rot, scale, opacity, color, sh_degree, cams, bg, rasterizer):
        scene = AnisoGaussianScene(pos.contiguous(), rot.contiguous(), scale.contiguous(), opacity.contiguous(),
                                   color.contiguous(), int(sh_degree))
        if len({(int(c.width), int(c.height)) for c in cams}) != 1:
            raise ValueError("AnisoGSRender: every camera must have the same size")
        images, st = rasterizer.render([scene] * len(cams), cams, bg, check="deferred", checkpoints=True, wide=True)
        if not any(ctx.needs_input_grad[:5]):
            rasterizer.verify(st)
        ctx.rasterizer, ctx.cams, ctx.bg, ctx.scene, ctx.st = rasterizer, cams, bg, scene, st
        out = st.pop("image").view(len(cams), 3, int(cams[0].height), int(cams[0].width))
        ctx.save_for_backward(out)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        st = ctx.st
        (image,) = ctx.saved_tensors
        g = ctx.rasterizer.render_bwd([ctx.scene] * len(ctx.cams), ctx.cams, st["fp"], st["bins"], ctx.bg,
                                      grad_out.contiguous().reshape(-1), st["T"], st["n_last"],
                                      image=image.reshape(-1), ckpt=st["ckpt"])[0]
        ctx.rasterizer.verify(st)
        return g.pos, g.rot, g.scale, g.opacity, g.color, None, None, None, None


__all__ = ["AnisoGaussianScene", "AnisoFootprints", "AnisoRasterizer", "AnisoGSRender"]
