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


def tile_outcomes(u, v, s, o, rgb, bins, view_id, width, bg=(0.0, 0.0, 0.0), pidx_offset=0, alpha_band=None,
                  term_band=None, pos_err=None, z32=None):
    """outcomes(y, x) -> (list of valid (C, T, n_last), resolved) of one pixel of a view, over
    its tile's list in ``bins`` (the oracle's ``pixel_outcomes``)."""
    TX = (int(width) + 15) // 16
    base = int(bins.tile_base[view_id])

    def fn(y, x):
        a, b = bins.ranges[base + (y // 16) * TX + x // 16]
        seq = bins.pidx[a:b].astype(np.int64) - pidx_offset
        return O.pixel_outcomes(x + 0.5, y + 0.5, seq, u, v, s, o, rgb, bg, alpha_band=alpha_band,
                                term_band=term_band, pos_err=pos_err, z32=z32)
    return fn


def f32_footprint_outcomes(views, bins, bg=(0.0, 0.0, 0.0), alpha_band=None, term_band=None):
    """tile_outcomes for each view of FP32 footprints (as given to the GPU stage tests)."""
    out, off = [], 0
    for vi, v in enumerate(views):
        with np.errstate(divide="ignore"):
            s = np.where(v["is2"] > 0, 1.0 / np.sqrt(v["is2"].astype(np.float64)), 1.0)
        out.append(tile_outcomes(v["u"].astype(np.float64), v["v"].astype(np.float64), s, v["o"].astype(np.float64),
                                 v["rgb"].astype(np.float64), bins, vi, v["width"], bg, off, alpha_band, term_band))
        off += v["u"].shape[0]
    return out


def projected_outcomes(projs, cams, bins, bg=(0.0, 0.0, 0.0), alpha_band=None, term_band=None):
    """tile_outcomes for each view of the oracle's FP64 projections, compared against
    footprints rounded elsewhere (centre errors and FP32 depths from footprint_uncertainty)."""
    out, off = [], 0
    for vi, (pr, cam) in enumerate(zip(projs, cams)):
        pe, z32 = O.footprint_uncertainty(pr)
        out.append(tile_outcomes(pr.u, pr.v, pr.s, pr.opacity, pr.rgb, bins, vi, cam.width, bg, off, alpha_band,
                                 term_band, pe, z32))
        off += pr.u.shape[0]
    return out


def check_image(gimg, gT, oimg, oT, flags, outcomes, tol=1e-4, max_flag_frac=0.01, what="", pixels=None):
    """Image parity with several correct results near a decision.

    gimg/oimg [3, H, W], gT/oT [H, W] (or, with ``pixels`` = (ys, xs), the same values at
    those pixels only: [3, P] and [P]). Unflagged pixels: colour and T within ``tol`` of the
    oracle's walk. Flagged pixels (at most ``max_flag_frac`` of them): within ``tol`` of at
    least one of the pixel's valid outcomes, every one of them resolved.
    Returns (max |d| unflagged, flagged count, max |d| to the nearest valid outcome)."""
    if pixels is None:
        H, W = flags.shape
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
        g = gimg.reshape(3, -1).astype(np.float64)
        gt = gT.reshape(-1).astype(np.float64)
        o, ot, fl = oimg.reshape(3, -1), oT.reshape(-1), flags.reshape(-1)
    else:
        ys, xs = pixels
        g, gt, o, ot, fl = gimg.astype(np.float64), gT.astype(np.float64), oimg, oT, flags
    d = np.maximum(np.abs(g - o).max(axis=0), np.abs(gt - ot))
    assert fl.mean() <= max_flag_frac, (what, "flagged fraction", float(fl.mean()), int(fl.sum()))
    worst_unflagged = float(d[~fl].max(initial=0.0))
    assert worst_unflagged <= tol, (what, worst_unflagged)
    worst_flagged = 0.0
    for p in np.nonzero(fl)[0]:
        outs, ok = outcomes(int(ys[p]), int(xs[p]))
        assert ok, (what, "unresolved pixel", int(ys[p]), int(xs[p]))
        best = min(max(float(np.abs(g[:, p] - c).max()), abs(float(gt[p]) - t)) for c, t, _ in outs)
        assert best <= tol, (what, "flagged pixel matches no valid outcome", int(ys[p]), int(xs[p]), best)
        worst_flagged = max(worst_flagged, best)
    return worst_unflagged, int(fl.sum()), worst_flagged


def grad_check(g_gpu, g_ref, name, rel=1e-3, floor=1e-4):
    """|GPU - oracle| <= rel |g| + floor max|g| for every element (no exemptions: the
    comparisons that use it give no weight to pixels where a decision is in band)."""
    a = np.asarray(g_gpu, dtype=np.float64)
    b = np.asarray(g_ref, dtype=np.float64)
    scale = float(np.abs(b).max())
    err = np.abs(a - b)
    bad = err > rel * np.abs(b) + floor * scale
    assert not bad.any(), (name, int(bad.sum()), bad.size, float(err.max()), scale)
    return float(err.max() / max(scale, 1e-30))


def split_flat(flat, cams, per_pixel_channels=3):
    out, off = [], 0
    for c in cams:
        n = per_pixel_channels * c.height * c.width
        a = flat[off:off + n]
        out.append(a.reshape(per_pixel_channels, c.height, c.width) if per_pixel_channels > 1
                   else a.reshape(c.height, c.width))
        off += n
    return out


# ---- anisotropic family ---------------------------------------------------------------------

def oracle_f32_aniso_footprints(projs, cams):
    """Per-view FP32 anisotropic footprints from the oracle's FP64 projection: the binning
    inputs of ``aniso64.f32_views_aniso`` plus the conic, opacity and colour."""
    out = []
    for pr, vw in zip(projs, O.aniso64.f32_views_aniso(projs, cams)):
        vis = pr.visible
        conic = np.array([np.where(vis, x, 0.0) for x in pr.conic]).astype(np.float32)
        out.append(dict(u=vw["u"], v=vw["v"], z=vw["z"], r=vw["r"], conic=conic,
                        o=np.where(vis, pr.opacity, 0.0).astype(np.float32),
                        rgb=np.where(vis[None, :], pr.rgb, 0.0).astype(np.float32),
                        width=vw["width"], height=vw["height"]))
    return out


def upload_aniso_footprints(views, bins, device="cuda"):
    """Packs per-view FP32 anisotropic footprints (+ the oracle's tile counts) into device
    AnisoFootprints: record {u, v, A, o, r, g, b, radius} and conic {B, C}."""
    import torch
    from paper_2403_14244_amd import AnisoFootprints, Footprints
    rec = np.concatenate([np.stack([v["u"], v["v"], v["conic"][0], v["o"], v["rgb"][0], v["rgb"][1], v["rgb"][2],
                                    v["r"]], 1) for v in views]).astype(np.float32)
    bc = np.concatenate([np.stack([v["conic"][1], v["conic"][2]], 1) for v in views]).astype(np.float32)
    z = np.concatenate([v["z"] for v in views]).astype(np.float32)
    tc = bins.tile_count.astype(np.int64).astype(np.int32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return AnisoFootprints(Footprints(t(rec), t(z), t(tc)), t(bc))


def oracle_aniso_render_f32(views, bins, bg=(0.0, 0.0, 0.0), q_err=None):
    """The oracle's tiled anisotropic render of FP32 footprints (upcast to FP64), per view."""
    res, off = [], 0
    for vi, v in enumerate(views):
        f64 = lambda a: np.asarray(a, dtype=np.float64)
        res.append(O.aniso64.render_aniso_tiled(f64(v["u"]), f64(v["v"]), f64(v["conic"]), f64(v["o"]),
                                                f64(v["rgb"]), bins, vi, v["width"], v["height"], bg,
                                                pidx_offset=off, q_err=q_err))
        off += v["u"].shape[0]
    return res


def aniso_outcomes(u, v, conic, o, rgb, bins, view_id, width, bg=(0.0, 0.0, 0.0), pidx_offset=0, q_err=None,
                   pos_err=None, z32=None):
    """outcomes(y, x) -> (valid results, resolved) of one pixel over its tile's list, for the
    anisotropic kernel (``aniso64.pixel_outcomes_aniso``)."""
    TX = (int(width) + 15) // 16
    base = int(bins.tile_base[view_id])

    def fn(y, x):
        a, b = bins.ranges[base + (y // 16) * TX + x // 16]
        seq = bins.pidx[a:b].astype(np.int64) - pidx_offset
        return O.aniso64.pixel_outcomes_aniso(x + 0.5, y + 0.5, seq, u, v, conic, o, rgb, bg, q_err=q_err,
                                              pos_err=pos_err, z32=z32)
    return fn
