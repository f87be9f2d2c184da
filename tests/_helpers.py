"""Shared test plumbing: oracle-side FP32 inputs for the per-stage GPU parity tests.

The stage tests feed BOTH sides the same FP32 inputs, produced by the oracle from a
seeded scene (never by the GPU path), so every difference is the stage's own.
"""
import numpy as np

import oracle as O


def oracle_f32_footprints(projs, cams):
    """Per-view FP32 footprints from the oracle's FP64 projection."""
    out = []
    for pr, vw in zip(projs, O.f32_views(projs, cams)):
        vis = pr.visible
        with np.errstate(all="ignore"):
            is2 = np.where(vis, 1.0 / (pr.s * pr.s), 0.0).astype(np.float32)
        out.append(dict(u=vw["u"], v=vw["v"], z=vw["z"], r=vw["r"], is2=is2,
                        o=np.where(vis, pr.opacity, 0.0).astype(np.float32),
                        rgb=np.where(vis[None, :], pr.rgb, 0.0).astype(np.float32),
                        width=vw["width"], height=vw["height"]))
    return out


def synthetic_f32_footprints(u, v, z, r, width, height, seed=0):
    """FP32 footprints for binning-only inputs (colour and kernel values are filler)."""
    rng = np.random.default_rng(seed)
    n = u.shape[0]
    return dict(u=u, v=v, z=z, r=r, is2=np.full(n, 0.25, np.float32),
                o=rng.uniform(0.1, 0.9, n).astype(np.float32),
                rgb=rng.uniform(0, 1, (3, n)).astype(np.float32), width=width, height=height)


def upload_footprints(views, bins, device="cuda"):
    """Packs per-view FP32 footprints (+ the oracle's tile counts) into device Footprints."""
    import torch
    from paper_2403_14244_amd import Footprints
    rec = np.concatenate([np.stack([v["u"], v["v"], v["is2"], v["o"], v["rgb"][0], v["rgb"][1], v["rgb"][2],
                                    v["r"]], 1) for v in views]).astype(np.float32)
    z = np.concatenate([v["z"] for v in views]).astype(np.float32)
    tc = bins.tile_count.astype(np.int64).astype(np.int32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return Footprints(t(rec), t(z), t(tc))


def upload_bins(b, capacity=None, device="cuda"):
    import torch
    from paper_2403_14244_amd import TileBins
    count = b.keys.shape[0]
    cap = max(count, 1) if capacity is None else capacity
    keys = np.zeros(cap, np.uint64)
    keys[:count] = b.keys
    pi = np.zeros(cap, np.uint32)
    pi[:count] = b.pidx
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(device)
    return TileBins(keys=t(keys, np.int64), pidx=t(pi, np.int32),
                    ranges=t(b.ranges, np.int32), offsets=t(b.offsets, np.int32),
                    count=torch.tensor([count], dtype=torch.int32, device=device),
                    status=torch.zeros(1, dtype=torch.int32, device=device), capacity=cap)


def oracle_render_f32(views, bins, bg=(0.0, 0.0, 0.0), tiles=None, alpha_band=None, term_band=None):
    """The oracle's tiled render of FP32 footprints (upcast to FP64), per view."""
    res = []
    off = 0
    for vi, v in enumerate(views):
        with np.errstate(divide="ignore"):
            s = np.where(v["is2"] > 0, 1.0 / np.sqrt(v["is2"].astype(np.float64)), 1.0)
        img, T, nl, fl = O.render64_tiled(v["u"].astype(np.float64), v["v"].astype(np.float64), s,
                                          v["o"].astype(np.float64), v["rgb"].astype(np.float64), bins, vi,
                                          v["width"], v["height"], bg, tiles=tiles, pidx_offset=off,
                                          with_flags=True, alpha_band=alpha_band, term_band=term_band)
        res.append((img, T, nl, fl))
        off += v["u"].shape[0]
    return res


def split_flat(flat, cams, per_pixel_channels=3):
    out, off = [], 0
    for c in cams:
        n = per_pixel_channels * c.height * c.width
        a = flat[off:off + n]
        out.append(a.reshape(per_pixel_channels, c.height, c.width) if per_pixel_channels > 1
                   else a.reshape(c.height, c.width))
        off += n
    return out
