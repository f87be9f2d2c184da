"""Torch-facing binding of the isotropic-splatting rasterizer.

PyTorch supplies device memory and the current HIP stream; every step of the pipeline
runs in the library's HIP kernels (see include/isogs.h for the contract of each call).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi as A

_F32 = torch.float32


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def sh_count(deg: int) -> int:
    return (deg + 1) ** 2


@dataclass
class GaussianScene:
    """Particle parameters on the device (FP32, structure of arrays).

    pos [3, N], scale [N] (sigma, linear), opacity [N] (activated), color [3K, N]."""
    pos: torch.Tensor
    scale: torch.Tensor
    opacity: torch.Tensor
    color: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.scale.shape[0])

    @staticmethod
    def from_host(scene, device="cuda") -> "GaussianScene":
        """From any object with numpy pos/scale/opacity/color/sh_degree (e.g. scenegen.Scene)."""
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return GaussianScene(t(scene.pos), t(scene.scale), t(scene.opacity), t(scene.color), int(scene.sh_degree))

    def validate(self):
        n = self.n
        K = sh_count(self.sh_degree)
        for name, x, shape in (("pos", self.pos, (3, n)), ("scale", self.scale, (n,)),
                               ("opacity", self.opacity, (n,)), ("color", self.color, (3 * K, n))):
            if tuple(x.shape) != shape or x.dtype != _F32 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError(f"scene.{name}: need a contiguous CUDA float32 tensor of shape {shape}")

    def abi(self) -> A.Scene:
        s = A.Scene()
        s.pos, s.scale, s.opacity, s.color = _p(self.pos), _p(self.scale), _p(self.opacity), _p(self.color)
        s.n = self.n
        s.sh_degree = self.sh_degree
        return s

    def empty_like(self) -> "GaussianScene":
        return GaussianScene(torch.empty_like(self.pos), torch.empty_like(self.scale),
                             torch.empty_like(self.opacity), torch.empty_like(self.color), self.sh_degree)

    def zeros_like(self) -> "GaussianScene":
        return GaussianScene(torch.zeros_like(self.pos), torch.zeros_like(self.scale),
                             torch.zeros_like(self.opacity), torch.zeros_like(self.color), self.sh_degree)


@dataclass
class Footprints:
    """Output of project: per (view, particle) records packed over views."""
    record: torch.Tensor         # [N, 8] {u, v, 1/s^2, o, r, g, b, radius}
    depth: torch.Tensor          # [N]
    tile_count: torch.Tensor     # [N] int32 (uint32 on the device)

    def abi(self) -> A.Projected:
        p = A.Projected()
        p.record, p.depth, p.tile_count = _p(self.record), _p(self.depth), _p(self.tile_count)
        return p

    @staticmethod
    def empty(n, device="cuda") -> "Footprints":
        return Footprints(torch.empty((n, 8), dtype=_F32, device=device), torch.empty(n, dtype=_F32, device=device),
                          torch.empty(n, dtype=torch.int32, device=device))


@dataclass
class TileBins:
    """Output of bin_sort. Entry arrays hold `capacity` slots; `count` and `status` live
    on the device, as the two adjacent words of one allocation (read back together)."""
    keys: torch.Tensor | None    # [capacity] int64 (uint64 on the device); None: not requested
    pidx: torch.Tensor           # [capacity] int32
    ranges: torch.Tensor         # [T, 2] int32
    offsets: torch.Tensor        # [N] int32
    count: torch.Tensor          # [1] int32
    status: torch.Tensor         # [1] int32
    capacity: int

    def abi(self) -> A.Bins:
        b = A.Bins()
        b.keys = _p(self.keys) if self.keys is not None else None
        b.pidx = _p(self.pidx)
        b.ranges, b.offsets = _p(self.ranges), _p(self.offsets)
        b.capacity = self.capacity
        b.count, b.status = _p(self.count), _p(self.status)
        return b

    def n_entries(self) -> int:
        return int(self.count.item())

    def verify(self):
        st = int(self.status.item())
        if st != A.ISOGS_OK:
            raise A.IsoGSError(st, f"bin_sort status {st} (entries {self.n_entries()}, capacity {self.capacity})")


def tiles_of(cam) -> int:
    return ((int(cam.width) + 15) // 16) * ((int(cam.height) + 15) // 16)


def _alloc_bins(capacity, n_total, tiles_total, device, with_keys=False) -> TileBins:
    cap = max(int(capacity), 1)
    words = torch.zeros(2, dtype=torch.int32, device=device)   # {count, status}: one fill, one read-back
    return TileBins(keys=torch.empty(cap, dtype=torch.int64, device=device) if with_keys else None,
                    pidx=torch.empty(cap, dtype=torch.int32, device=device),
                    ranges=torch.empty((tiles_total, 2), dtype=torch.int32, device=device),
                    offsets=torch.empty(max(n_total, 1), dtype=torch.int32, device=device)[:n_total],
                    count=words[0:1], status=words[1:2], capacity=cap)


class Rasterizer:
    """Runs project -> bin_sort -> render_fwd (and render_bwd) through the C ABI, keeping
    workspaces and the entry capacity between calls. The capacity grows on demand: when a
    bin_sort reports overflow it is re-run once with the exact count plus headroom."""

    def __init__(self, device="cuda", headroom=1.25):
        self.device = torch.device(device)
        self.headroom = headroom
        self.capacity = 0
        self.ordered_fwd = True
        # sync_free: IsoGSRender reads no capacity status at all (not even deferred), so a
        # training step can be captured in a HIP graph; the capacity must be sized first
        # (an eager step), and a pass that overflows it shows NaN images and loss
        self.sync_free = False
        self._ws = torch.empty(0, dtype=torch.uint8, device=self.device)

    def _workspace(self, nbytes):
        if self._ws.numel() < nbytes:
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return self._ws

    # -- the four ABI calls -----------------------------------------------------------
    def project(self, scenes, cams) -> Footprints:
        n_total = sum(s.n for s in scenes)
        fp = Footprints.empty(n_total, self.device)
        sc = (A.Scene * len(scenes))(*[s.abi() for s in scenes])
        A.check(A.lib().isogs_project(sc, A.camera_array(cams), len(cams), ctypes.byref(fp.abi()), _stream()))
        return fp

    def bin_sort(self, fp: Footprints, n_per_view, cams, check=True, capacity=None, with_keys=False) -> TileBins:
        """Bins and sorts the entries. The 64-bit (tile, depth) keys are written only with
        `with_keys` (compositing needs pidx and the tile ranges alone)."""
        npv = A.int_array(n_per_view)
        carr = A.camera_array(cams)
        n_total = int(sum(n_per_view))
        tiles_total = sum(tiles_of(c) for c in cams)
        cap = self.capacity if capacity is None else capacity
        for _ in range(2):
            bins = _alloc_bins(cap, n_total, tiles_total, self.device, with_keys)
            ab = bins.abi()
            need = ctypes.c_size_t(0)
            A.check(A.lib().isogs_bin_sort(ctypes.byref(fp.abi()), npv, carr, len(cams), ctypes.byref(ab), None,
                                           ctypes.byref(need), _stream()))
            ws = self._workspace(need.value)
            have = ctypes.c_size_t(ws.numel())
            A.check(A.lib().isogs_bin_sort(ctypes.byref(fp.abi()), npv, carr, len(cams), ctypes.byref(ab),
                                           _p(ws), ctypes.byref(have), _stream()))
            if not check:
                return bins
            st = int(bins.status.item())
            if st == A.ISOGS_OK:
                return bins
            if st != A.ISOGS_ERR_CAPACITY:
                raise A.IsoGSError(st, "bin_sort failed on the device")
            cap = int(bins.n_entries() * self.headroom) + 4096
            if capacity is None:
                self.capacity = cap
        raise A.IsoGSError(A.ISOGS_ERR_CAPACITY, "bin_sort capacity still too small after growing")

    def bin_sort_static(self, fp: Footprints, n_per_view, cams, capacity, with_keys=False) -> TileBins:
        """bin_sort through isogs_bin_sort_static: the library's scratch is its static
        per-GPU array, so the only allocations are the output bins made here (a caller
        that cannot allocate passes bins it made beforehand to the C call). No capacity
        retry: the status is left on the device for the caller."""
        bins = _alloc_bins(capacity, int(sum(n_per_view)), sum(tiles_of(c) for c in cams), self.device, with_keys)
        A.check(A.lib().isogs_bin_sort_static(ctypes.byref(fp.abi()), A.int_array(n_per_view), A.camera_array(cams),
                                              len(cams), ctypes.byref(bins.abi()), _stream()))
        return bins

    def checkpoint_buffer(self, bins: TileBins) -> torch.Tensor:
        """Device buffer for the compositing checkpoints of these bins (see render_bwd)."""
        nbytes = int(A.lib().isogs_checkpoint_bytes(bins.capacity))
        return torch.empty(nbytes // 4, dtype=_F32, device=self.device)

    def render_fwd(self, fp: Footprints, n_per_view, bins: TileBins, cams, bg=(0.0, 0.0, 0.0), ckpt=None,
                   last=True):
        """Composites every view; with `ckpt` (from checkpoint_buffer) also stores the
        checkpoints that let render_bwd split long tiles. `last=False`: no n_last (None),
        for a forward that no backward pass follows."""
        pix = sum(int(c.width) * int(c.height) for c in cams)
        image = torch.empty(3 * pix, dtype=_F32, device=self.device)
        T = torch.empty(pix, dtype=_F32, device=self.device)
        n_last = torch.empty(pix, dtype=torch.int32, device=self.device) if last else None
        bgc = (ctypes.c_float * 3)(*[float(b) for b in bg])
        A.check(A.lib().isogs_render_fwd(ctypes.byref(fp.abi()), A.int_array(n_per_view), ctypes.byref(bins.abi()),
                                         A.camera_array(cams), len(cams), bgc, _p(image), _p(T), _p(n_last),
                                         _p(ckpt), _stream()))
        return image, T, n_last

    def render_fwd_ordered(self, fp: Footprints, n_per_view, bins: TileBins, cams, bg=(0.0, 0.0, 0.0),
                           out=None, ckpt=None, wide=False, times=False, last=True):
        """render_fwd with the tiles dispatched longest entry list first (same result).
        `wide`: the longest tiles of small launches are composited four lanes per pixel
        (same result up to rounding on those tiles; about twice as fast for one view).
        `out` optionally supplies (image, T_final, n_last) buffers (n_last may be None).
        `last=False`: no n_last (None), for a forward that no backward pass follows (the
        walk then skips tracking the last entry). `times`: also returns the per-workgroup
        {start, end} stamps of the 100 MHz clock, int64 [5 * tiles, 2] ({0, 0} for
        workgroups without a non-empty list), as a view of the workspace that the next call
        on this rasterizer overwrites."""
        pix = sum(int(c.width) * int(c.height) for c in cams)
        if out is None:
            out = (torch.empty(3 * pix, dtype=_F32, device=self.device),
                   torch.empty(pix, dtype=_F32, device=self.device),
                   torch.empty(pix, dtype=torch.int32, device=self.device) if last else None)
        image, T, n_last = out
        bgc = (ctypes.c_float * 3)(*[float(b) for b in bg])
        carr = A.camera_array(cams)
        npv = A.int_array(n_per_view)
        need = ctypes.c_size_t(0)
        flags = (A.ISOGS_FWD_WIDE if wide else 0) | (A.ISOGS_FWD_TIMES if times else 0)
        args = (ctypes.byref(fp.abi()), npv, ctypes.byref(bins.abi()), carr, len(cams), bgc, _p(image), _p(T),
                _p(n_last), _p(ckpt), flags)
        A.check(A.lib().isogs_render_fwd_ordered(*args, None, ctypes.byref(need), _stream()))
        ws = self._workspace_q(need.value)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_render_fwd_ordered(*args, _p(ws), ctypes.byref(have), _stream()))
        if not times:
            return image, T, n_last
        base = ctypes.c_size_t(0)
        A.check(A.lib().isogs_render_fwd_ordered(*args[:-1], flags & ~A.ISOGS_FWD_TIMES, None, ctypes.byref(base),
                                                 _stream()))
        tiles = sum(((int(c.width) + 15) // 16) * ((int(c.height) + 15) // 16) for c in cams)
        off = base.value - 256
        stamps = ws[off:off + tiles * 5 * 16].view(torch.int64).view(tiles * 5, 2)
        return image, T, n_last, stamps

    def _workspace_q(self, nbytes):
        if not hasattr(self, "_wsq") or self._wsq.numel() < nbytes:
            self._wsq = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return self._wsq

    def render_bwd(self, scenes, cams, fp: Footprints, bins: TileBins, bg, dL_dimage, T_final, n_last, grads=None,
                   image=None, ckpt=None):
        """Returns one GaussianScene of gradients per distinct scene (by pos pointer), in
        order of first appearance; views of one scene are summed. With the forward's image
        and checkpoints, long tiles are walked as chunks on several workgroups."""
        if grads is None:
            uniq = {}
            for s in scenes:
                if s.pos.data_ptr() not in uniq:
                    uniq[s.pos.data_ptr()] = s.empty_like()   # the library overwrites every output
            grads = [uniq[s.pos.data_ptr()] for s in scenes]
        sc = (A.Scene * len(scenes))(*[s.abi() for s in scenes])
        gs = (A.Scene * len(scenes))(*[g.abi() for g in grads])
        bgc = (ctypes.c_float * 3)(*[float(b) for b in bg])
        need = ctypes.c_size_t(0)
        ab = bins.abi()
        args = (sc, A.camera_array(cams), len(cams), ctypes.byref(fp.abi()), ctypes.byref(ab), bgc, _p(image),
                _p(dL_dimage.contiguous()), _p(T_final), _p(n_last), _p(ckpt), gs)
        A.check(A.lib().isogs_render_bwd(*args, None, ctypes.byref(need), _stream()))
        ws = self._workspace(need.value)
        have = ctypes.c_size_t(ws.numel())
        A.check(A.lib().isogs_render_bwd(*args, _p(ws), ctypes.byref(have), _stream()))
        out, seen = [], set()
        for g in grads:
            if g.pos.data_ptr() not in seen:
                seen.add(g.pos.data_ptr())
                out.append(g)
        return out

    # -- convenience ------------------------------------------------------------------
    def render(self, scenes, cams, bg=(0.0, 0.0, 0.0), check=True, checkpoints=False, wide=False):
        """Full forward pass. Returns (list of [3, H, W] images, state for backward).

        `check=True`: everything is queued before the one host synchronisation that the
        capacity status needs; on overflow the capacity grows and the pass is redone.
        `check="deferred"`: once a capacity is known, nothing waits: the status is copied
        to pinned host memory behind the launches and `verify(state)` reads it later (the
        first call, with no capacity yet, still checks synchronously); until then, an
        overflowed pass shows NaN images and transmittance (the library's compositing
        writes NaN when the bins overflowed). With
        `ordered_fwd` set, compositing dispatches the tiles longest list first
        (same images bitwise; with `wide`, the longest tiles of small launches are
        composited four lanes per pixel, equal up to rounding). `checkpoints` keeps the
        compositing checkpoints for the backward in the state."""
        fp = self.project(scenes, cams)
        npv = [s.n for s in scenes]
        if self.ordered_fwd:
            fwd = lambda *a, **k: self.render_fwd_ordered(*a, wide=wide, **k)
        else:
            fwd = self.render_fwd
        bins = self.bin_sort(fp, npv, cams, check=False)
        ckpt = self.checkpoint_buffer(bins) if checkpoints else None
        out = fwd(fp, npv, bins, cams, bg, ckpt=ckpt)
        pending = None
        if check == "deferred" and self.capacity > 0:
            pending = torch.empty(2, dtype=torch.int32, pin_memory=True)
            # count and status are adjacent words of one allocation (_alloc_bins): one copy
            pending.copy_(bins.count.as_strided((2,), (1,)), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream())
            pending = (pending, ev)
        elif check:
            st = int(bins.status.item())
            if st == A.ISOGS_ERR_CAPACITY:
                self.capacity = int(bins.n_entries() * self.headroom) + 4096
                bins = self.bin_sort(fp, npv, cams, check=True)
                ckpt = self.checkpoint_buffer(bins) if checkpoints else None
                out = fwd(fp, npv, bins, cams, bg, ckpt=ckpt)
            elif st != A.ISOGS_OK:
                raise A.IsoGSError(st, "bin_sort failed on the device")
        image, T, n_last = out
        return split_images(image, cams), dict(fp=fp, bins=bins, image=image, T=T, n_last=n_last, npv=npv,
                                               pending=pending, ckpt=ckpt)

    def verify(self, state):
        """Reads a deferred status (waiting for the forward launches if needed). On a
        capacity overflow the capacity grows for the next call and IsoGSError is raised:
        that pass's outputs are not valid."""
        if state.get("pending") is None:
            return
        host, ev = state["pending"]
        ev.synchronize()
        count, st = int(host[0]), int(host[1])   # {count, status}
        state["pending"] = None
        if st == A.ISOGS_ERR_CAPACITY:
            self.capacity = int(count * self.headroom) + 4096
            raise A.IsoGSError(st, f"entry capacity overflowed in the forward pass ({count} entries); "
                                   f"capacity grown to {self.capacity}, repeat the pass")
        if st != A.ISOGS_OK:
            raise A.IsoGSError(st, "bin_sort failed on the device")


def split_images(flat, cams):
    out, off = [], 0
    for c in cams:
        h, w = int(c.height), int(c.width)
        out.append(flat[off:off + 3 * h * w].view(3, h, w))
        off += 3 * h * w
    return out


class IsoGSRender(torch.autograd.Function):
    """Differentiable render of one scene from V cameras of equal size.

    forward(pos, scale, opacity, color, sh_degree, cams, bg, rasterizer) -> [V, 3, H, W].
    Parameters are the activated values (sigma > 0, o in (0, 1)); gradients flow to all
    four parameter tensors; views are summed in order by the library."""

    @staticmethod
    def forward(ctx, pos, scale, opacity, color, sh_degree, cams, bg, rasterizer):
        scene = GaussianScene(pos.contiguous(), scale.contiguous(), opacity.contiguous(), color.contiguous(),
                              int(sh_degree))
        scenes = [scene] * len(cams)
        if len({(int(c.width), int(c.height)) for c in cams}) != 1:
            raise ValueError("IsoGSRender: every camera must have the same size")
        check = False if rasterizer.sync_free else "deferred"
        images, st = rasterizer.render(scenes, cams, bg, check=check, checkpoints=True, wide=True)
        if not any(ctx.needs_input_grad[:4]):
            # no backward will read the deferred status: read it now (an overflowed pass
            # raises here; its images are NaN, never silently stale)
            rasterizer.verify(st)
        ctx.rasterizer = rasterizer
        ctx.cams = cams
        ctx.bg = bg
        ctx.scene = scene
        ctx.st = st
        # the views are packed back to back in one buffer: the batch is a view of it, no
        # copy. The backward reads the same buffer (checkpointed tiles restart from it), so
        # it is saved as an output: autograd then refuses a backward after an in-place
        # change of the returned images.
        out = st.pop("image").view(len(cams), 3, int(cams[0].height), int(cams[0].width))
        ctx.save_for_backward(out)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        st = ctx.st
        (image,) = ctx.saved_tensors
        scenes = [ctx.scene] * len(ctx.cams)
        g = ctx.rasterizer.render_bwd(scenes, ctx.cams, st["fp"], st["bins"], ctx.bg,
                                      grad_out.contiguous().reshape(-1), st["T"], st["n_last"],
                                      image=image.reshape(-1), ckpt=st["ckpt"])[0]
        # the forward's capacity status is read only now, behind the queued backward, so
        # that neither pass waits for the device (on an overflow every kernel after the
        # sort skipped its work and this raises)
        ctx.rasterizer.verify(st)
        return g.pos, g.scale, g.opacity, g.color, None, None, None, None
