"""FP64 CPU oracle of the anisotropic variant of the splatting path.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never calls it
and shares no code, constants table or helper with it.

The paper (Gong, Yu, Yue, arXiv 2403.14244) sets its isotropic kernel against the
anisotropic Gaussians of 3D Gaussian splatting, which Section 1 states as:

* eq. 5, the kernel G(x) = exp(-(x - mu)^T Sigma^-1 (x - mu)) (no factor 1/2, as in eq. 8);
* eq. 6, the covariance Sigma = R S S^T R^T from a rotation R and a scaling S;
* eq. 7, its screen-space covariance Sigma_2D = J V Sigma V^T J^T, with V the view
  transformation and J the Jacobian of the affine approximation of the projection.

Readings taken here (the paper is silent on them):

* R is the rotation of the unit quaternion q / |q|, q = (w, x, y, z) stored per particle;
  S = diag(s1, s2, s3) with linear world-space scales, so Sigma = R diag(s^2) R^T;
* V is the rotation part of the camera (p = V mu + t) and J the Jacobian of the pinhole
  map (p_x, p_y, p_z) -> (f p_x / p_z + cx, f p_y / p_z + cy) at the particle's centre,
  J = [[f/z, 0, -f p_x / z^2], [0, f/z, -f p_y / z^2]]; no low-pass term is added to
  Sigma_2D (eq. 7 has none);
* the screen kernel is eq. 5 with Sigma_2D: G = exp(-(A dx^2 + 2 B dx dy + C dy^2)) where
  [[A, B], [B, C]] = Sigma_2D^-1 (the conic) and (dx, dy) the pixel centre minus the
  projected centre; alpha = min(0.99, o G) and everything after it (the 1/255 support, the
  front-to-back compositing of eq. 4, the stop at T < 1e-4, the tiles and the depth order)
  is the isotropic path's;
* the binning radius is that of the disk around the support ellipse A dx^2 + 2 B dx dy +
  C dy^2 <= ln(255 o): sqrt(lambda_max(Sigma_2D) ln(255 o)), grown as the isotropic radius
  is, so that the tile lists stay a superset of the support.

With Sigma = sigma^2 I the screen covariance is sigma^2 J J^T (the full projection of an
isotropic Gaussian); on the optical axis it is the circle of scale f sigma / z that the
isotropic path uses.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import isogs64 as I


@dataclass
class AnisoProjected64:
    """FP64 screen footprints of one view."""
    u: np.ndarray
    v: np.ndarray
    z: np.ndarray
    cov: np.ndarray        # [3, n]: a, b, c of Sigma_2D = [[a, b], [b, c]]
    conic: np.ndarray      # [3, n]: A, B, C of Sigma_2D^-1 = [[A, B], [B, C]]
    opacity: np.ndarray
    rgb: np.ndarray        # [3, n], clamped at 0
    radius: np.ndarray     # binning radius (pixels); 0 where not visible
    visible: np.ndarray
    # kept for the backward pass
    p: np.ndarray          # camera-space centre [3, n]
    rotm: np.ndarray       # [3, 3, n] rotation of the normalised quaternion
    qnorm: np.ndarray      # |q|
    dirs: np.ndarray
    dist: np.ndarray
    rgb_raw: np.ndarray


def quat_to_rot(q):
    """Rotation matrices [3, 3, n] of the unit quaternions q [4, n] = (w, x, y, z): the
    rotation by angle theta about the unit axis a is (cos(theta/2), sin(theta/2) a).
    Pinned: orthonormal with determinant 1, q and -q give the same matrix, and the
    quaternion of a rotation about z by theta gives the textbook matrix."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def covariance3d(rotm, scale):
    """Sigma = R S S^T R^T (eq. 6) for each particle: [3, 3, n]."""
    M = rotm * scale[None, :, :]                    # R S (columns scaled)
    return np.einsum("ikn,jkn->ijn", M, M)


def screen_jacobian(p, f):
    """Jacobian [2, 3, n] of (p_x, p_y, p_z) -> (f p_x / p_z, f p_y / p_z) at p [3, n]."""
    z = p[2]
    zero = np.zeros_like(z)
    return np.array([[f / z, zero, -f * p[0] / (z * z)],
                     [zero, f / z, -f * p[1] / (z * z)]])


def project_aniso64(scene, cam) -> AnisoProjected64:
    """Footprint of every particle in one view (eq. 6, eq. 7), FP64 from the FP32 inputs.
    ``scene`` has pos [3, n], rot [4, n] (quaternions w, x, y, z), scale [3, n] (linear,
    per axis), opacity [n], color [3K, n] and sh_degree.

    p = V mu + t, z = p_z; u = f p_x / z + cx, v = f p_y / z + cy; Sigma_2D = T Sigma T^T
    with T = J V; conic = Sigma_2D^-1; colour as in the isotropic path. A particle is
    invisible when any input is non-finite, a scale is <= 0, |q| = 0, o < 1/255, z <= near,
    det Sigma_2D <= 0, or its footprint has no normal FP32 form (the centre, the conic or
    the binning radius overflowing, A or C below the smallest normal FP32 value).
    Pinned by the isotropic closed forms (on the axis the conic is I / s^2 with
    s = f sigma / z), by a finite-difference Jacobian of the pinhole map, by the swap of
    A and C under a quarter turn about the optical axis, and by finite differences of the
    rendered image."""
    V, t, eye, f, cx, cy, near = I._cam64(cam)
    mu = scene.pos.astype(np.float64)
    q = scene.rot.astype(np.float64)
    sc = scene.scale.astype(np.float64)
    o = scene.opacity.astype(np.float64)
    coef = scene.color.astype(np.float64)
    n = o.shape[0]
    K = I.sh_count(scene.sh_degree)
    with np.errstate(all="ignore"):
        qn = np.sqrt((q * q).sum(axis=0))
        qh = q / qn
        rotm = quat_to_rot(qh)
        Sig = covariance3d(rotm, sc)
        p = V @ mu + t[:, None]
        z = p[2]
        u = f * p[0] / z + cx
        v = f * p[1] / z + cy
        J = screen_jacobian(p, f)
        T = np.einsum("ikn,kj->ijn", J, V)             # J V  [2, 3, n]
        cov2 = np.einsum("ikn,kln,jln->ijn", T, Sig, T)
        a, b, c = cov2[0, 0], cov2[0, 1], cov2[1, 1]
        det = a * c - b * b
        A, B, C = c / det, -b / det, a / det
        lam = 0.5 * (a + c) + np.sqrt(0.25 * (a - c) ** 2 + b * b)
        dvec = mu - eye[:, None]
        dist = np.sqrt((dvec * dvec).sum(axis=0))
        dirs = dvec / dist
        basis = I.sh_basis(scene.sh_degree, dirs)
        c3 = coef.reshape(K, 3, n)
        rgb_raw = c3[0].copy()
        for k in range(1, K):
            rgb_raw = rgb_raw + c3[k] * basis[k]
        rgb = np.maximum(rgb_raw, 0.0)
        finite = (np.isfinite(mu).all(axis=0) & np.isfinite(q).all(axis=0) & np.isfinite(sc).all(axis=0)
                  & np.isfinite(o) & np.isfinite(coef).all(axis=0))
        visible = finite & (sc > 0).all(axis=0) & (qn > 0) & (o >= I.ALPHA_MIN) & (z > near)
        visible &= np.isfinite(u) & np.isfinite(v) & np.isfinite(det) & (det > 0) & np.isfinite(rgb).all(axis=0)
        radius = np.where(visible, np.sqrt(lam * np.log(np.where(visible, 255.0 * o, 1.0))) * I.RADIUS_GROW
                          + I.RADIUS_PAD, 0.0)
        tiny = np.finfo(np.float32).tiny
        A32, B32, C32 = (np.where(visible, x, 1.0).astype(np.float32) for x in (A, B, C))
        visible &= (np.isfinite(A32) & np.isfinite(B32) & np.isfinite(C32) & (A32 >= tiny) & (C32 >= tiny)
                    & np.isfinite(radius.astype(np.float32)) & np.isfinite(u.astype(np.float32))
                    & np.isfinite(v.astype(np.float32)))
        radius = np.where(visible, radius, 0.0)
    return AnisoProjected64(u=u, v=v, z=z, cov=np.array([a, b, c]), conic=np.array([A, B, C]), opacity=o,
                            rgb=rgb, radius=radius, visible=visible, p=p, rotm=rotm, qnorm=qn, dirs=dirs,
                            dist=dist, rgb_raw=rgb_raw)


# --------------------------------------------------------------------------------------
# Compositing (eq. 4) with the anisotropic kernel (eq. 5).
# --------------------------------------------------------------------------------------

def kernel_exponent(dx, dy, conic_g):
    """A dx^2 + 2 B dx dy + C dy^2 for one particle's conic (A, B, C)."""
    A, B, C = conic_g
    return A * dx * dx + 2.0 * B * dx * dy + C * dy * dy


def centre_growth(dx, dy, conic_g, e):
    """Largest change of Q = d^T M d (M the conic) when the centre moves by at most e in x
    and in y: 2 (|(M d)_x| + |(M d)_y|) e + (|A| + 2 |B| + |C|) e^2. For a circle M = I / s^2
    this is the isotropic walk's bound (2 (|dx| + |dy|) e + 2 e^2) / s^2."""
    A, B, C = conic_g
    return (2.0 * (np.abs(A * dx + B * dy) + np.abs(B * dx + C * dy)) * e
            + (abs(A) + 2.0 * abs(B) + abs(C)) * e * e)


def composite_pixels_aniso(px, py, seq, u, v, conic, o, rgb, bg, trace=False, alpha_band=None, term_band=None,
                           q_err=None, pos_err=None, z32=None):
    """Front-to-back compositing (eq. 4) of one particle sequence at a set of pixel centres
    with the kernel of eq. 5: G = exp(-(A dx^2 + 2 B dx dy + C dy^2)), alpha = min(0.99, o G),
    an entry is skipped when alpha < 1/255, C += c alpha T, T *= 1 - alpha, the pixel stops
    after T < 1e-4; finally C += T bg. Returns (C [3, P], T_final [P], n_last [P]) and with
    ``trace`` the flags of pixels near a decision: some alpha within a relative
    ``alpha_band`` (plus ``q_err`` times |A| dx^2 + 2 |B dx dy| + |C| dy^2, the uncertainty of an
    exponent evaluated in lower precision) of 1/255, or some T after an entry within a
    relative ``term_band`` (grown by what those alpha uncertainties can do to T) of 1e-4.
    Pinned: equal to the isotropic walk for circular conics, tiled == untiled, finite
    differences of its gradients.

    For footprints that are the FP32 roundings of these (an end-to-end comparison),
    ``pos_err`` [n] bounds each centre's error (the alpha band grows by ``centre_growth``,
    and the band of T by what that does to T, as in ``isogs64.composite_pixels``) and
    ``z32`` [n] gives the FP32 depths: two consecutive composited entries at most one ulp
    apart flag the pixel (their order may differ)."""
    alpha_band = I.ALPHA_FLAG_REL if alpha_band is None else alpha_band
    term_band = I.TERM_FLAG_REL if term_band is None else term_band
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    P = px.shape[0]
    T = np.ones(P)
    C = np.zeros((3, P))
    n_last = np.zeros(P, dtype=np.int64)
    done = np.zeros(P, dtype=bool)
    near_alpha = np.zeros(P, dtype=bool)
    near_term = np.zeros(P, dtype=bool)
    t_band = np.full(P, float(term_band))
    zb = None if z32 is None else np.asarray(z32, dtype=np.float32).view(np.int32).astype(np.int64)
    prev_z = np.full(P, -(1 << 40), dtype=np.int64)
    rec = [] if trace else None
    for pos, g in enumerate(seq):
        if done.all():
            break
        dx = px - u[g]
        dy = py - v[g]
        Q = kernel_exponent(dx, dy, conic[:, g])
        G = np.exp(-Q)
        a = np.minimum(I.ALPHA_MAX, o[g] * G)
        live = ~done
        grow = 0.0
        if q_err is not None:
            A, B, Cc = conic[:, g]
            grow = q_err * (abs(A) * dx * dx + 2.0 * abs(B) * np.abs(dx * dy) + abs(Cc) * dy * dy)
        if pos_err is not None:
            grow = grow + centre_growth(dx, dy, conic[:, g], float(pos_err[g]))
        near_alpha |= live & (np.abs(a * 255.0 - 1.0) <= alpha_band + grow)
        use = live & (a >= I.ALPHA_MIN)
        if not use.any():
            continue
        w = np.where(use, a * T, 0.0)
        C = C + rgb[:, g][:, None] * w[None, :]
        T_new = np.where(use, T * (1.0 - a), T)
        t_band = t_band + np.where(use, a / (1.0 - a) * grow, 0.0)
        near_term |= use & (np.abs(T_new / I.T_MIN - 1.0) <= t_band)
        if zb is not None:
            near_alpha |= use & (np.abs(zb[g] - prev_z) <= 1)
            prev_z = np.where(use, zb[g], prev_z)
        if trace:
            rec.append((pos, g, np.where(use, a, 0.0), T.copy(), use.copy(), G))
        T = T_new
        n_last = np.where(use, pos + 1, n_last)
        done |= use & (T < I.T_MIN)
    C = C + T[None, :] * np.asarray(bg, dtype=np.float64)[:, None]
    if trace:
        return C, T, n_last, dict(records=rec, near_alpha=near_alpha, near_term=near_term)
    return C, T, n_last


def pixel_outcomes_aniso(px, py, seq, u, v, conic, o, rgb, bg=(0.0, 0.0, 0.0), alpha_band=None, term_band=None,
                         q_err=None, slack=1e-5, max_branch=12, pos_err=None, z32=None):
    """Every valid result of one pixel near a decision (``isogs64.pixel_outcomes``) for the
    kernel of eq. 5, the alpha bands grown as in ``composite_pixels_aniso`` (with ``z32``, the
    order of two entries one FP32 ulp apart in depth is also taken both ways)."""
    seq = np.asarray(seq, dtype=np.int64)
    dx = float(px) - u[seq]
    dy = float(py) - v[seq]
    cg = conic[:, seq]
    Q = cg[0] * dx * dx + 2.0 * cg[1] * dx * dy + cg[2] * dy * dy
    a = np.minimum(I.ALPHA_MAX, o[seq] * np.exp(-Q))
    grow = np.zeros(seq.shape[0])
    if q_err is not None:
        grow = q_err * (np.abs(cg[0]) * dx * dx + 2.0 * np.abs(cg[1] * dx * dy) + np.abs(cg[2]) * dy * dy)
    if pos_err is not None:
        grow = grow + centre_growth(dx, dy, cg, np.asarray(pos_err, dtype=np.float64)[seq])
    zs = None if z32 is None else np.asarray(z32, dtype=np.float32)[seq]
    return I.walk_outcomes(a, grow, rgb[:, seq], bg, alpha_band, term_band, zs, slack, max_branch)


def f32_views_aniso(projs, cams):
    """FP32 binning inputs (u, v, z, r) of anisotropic footprints, one dict per view."""
    out = []
    for pr, cam in zip(projs, cams):
        out.append(dict(u=np.where(pr.visible, pr.u, 0.0).astype(np.float32),
                        v=np.where(pr.visible, pr.v, 0.0).astype(np.float32),
                        z=np.where(pr.visible, pr.z, 1.0).astype(np.float32),
                        r=np.where(pr.visible, pr.radius, 0.0).astype(np.float32),
                        width=cam.width, height=cam.height))
    return out


def depth_order_aniso(proj: AnisoProjected64):
    idx = np.nonzero(proj.visible)[0]
    return idx[np.lexsort((idx, proj.z[idx]))]


def render_aniso_untiled(proj: AnisoProjected64, width, height, bg=(0.0, 0.0, 0.0)):
    """The plain definition: every pixel walks every visible particle in depth order."""
    seq = depth_order_aniso(proj)
    X, Y = np.meshgrid(np.arange(width), np.arange(height))
    C, T, _ = composite_pixels_aniso(X.ravel() + 0.5, Y.ravel() + 0.5, seq, proj.u, proj.v, proj.conic,
                                     proj.opacity, proj.rgb, bg)
    return C.reshape(3, height, width), T.reshape(height, width)


def render_aniso_tiled(u, v, conic, o, rgb, bins, view_id, width, height, bg=(0.0, 0.0, 0.0), pidx_offset=0,
                       q_err=None, tiles=None, pos_err=None, z32=None):
    """Per-tile rendering of one view over the lists of ``isogs64.bin_sort_ref``. Returns
    image [3, H, W], T_final [H, W], n_last [H, W] and the flags [H, W]."""
    TX, TY = I.tile_grid(width, height)
    img = np.zeros((3, height, width))
    Tf = np.ones((height, width))
    nl = np.zeros((height, width), dtype=np.int64)
    flags = np.zeros((height, width), dtype=bool)
    base = int(bins.tile_base[view_id])
    tiles = [(tx, ty) for ty in range(TY) for tx in range(TX)] if tiles is None else tiles
    for tx, ty in tiles:
        a, b = bins.ranges[base + ty * TX + tx]
        seq = bins.pidx[a:b].astype(np.int64) - pidx_offset
        X, Y = I.tile_pixels(tx, ty, width, height)
        C, T, n, tr = composite_pixels_aniso(X + 0.5, Y + 0.5, seq, u, v, conic, o, rgb, bg, trace=True,
                                             q_err=q_err, pos_err=pos_err, z32=z32)
        img[:, Y, X] = C
        Tf[Y, X] = T
        nl[Y, X] = n
        flags[Y, X] = tr["near_alpha"] | tr["near_term"]
    return img, Tf, nl, flags


def render_aniso_views(scenes, cams, bg=(0.0, 0.0, 0.0), q_err=None, rounded=False, tiles=None):
    """Projects, bins and renders each (scene, camera) pair with the tiled oracle. Returns
    (images, T_final, n_last, flags, projections, bins), lists over the views. ``rounded``:
    the flags allow for footprints rounded once to FP32 elsewhere (centre errors and FP32
    depths from ``isogs64.footprint_uncertainty``)."""
    projs = [project_aniso64(sc, cam) for sc, cam in zip(scenes, cams)]
    bins = I.bin_sort_ref(f32_views_aniso(projs, cams))
    out = ([], [], [], [])
    off = 0
    for vi, (pr, cam) in enumerate(zip(projs, cams)):
        pe, z32 = I.footprint_uncertainty(pr) if rounded else (None, None)
        res = render_aniso_tiled(pr.u, pr.v, pr.conic, pr.opacity, pr.rgb, bins, vi, cam.width, cam.height, bg,
                                 pidx_offset=off, q_err=q_err, tiles=tiles, pos_err=pe, z32=z32)
        for lst, x in zip(out, res):
            lst.append(x)
        off += pr.u.shape[0]
    return (*out, projs, bins)


# --------------------------------------------------------------------------------------
# Backward.
# --------------------------------------------------------------------------------------

def composite_backward_aniso(px, py, seq, u, v, conic, o, rgb, bg, dC):
    """Gradient of L = sum_p <dC[:, p], C_p> with respect to each entry's screen parameters.

    dC/dc_k and dC/dalpha_k as in the isotropic walk (eq. 4); below the clamp,
    alpha = o exp(-Q) with Q = A dx^2 + 2 B dx dy + C dy^2 and dx = x - u, dy = y - v:
      dalpha/du = alpha (2 A dx + 2 B dy), dalpha/dv = alpha (2 B dx + 2 C dy),
      dalpha/dA = -alpha dx^2, dalpha/dB = -2 alpha dx dy, dalpha/dC = -alpha dy^2,
      dalpha/do = alpha / o.
    Returns per-particle sums: du, dv, dA, dB, dC, do, drgb [3]. Pinned by central finite
    differences of ``composite_pixels_aniso``."""
    _, T, _, tr = composite_pixels_aniso(px, py, seq, u, v, conic, o, rgb, bg, trace=True)
    S = T[None, :] * np.asarray(bg, dtype=np.float64)[:, None]
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    out = {}
    for pos, g, a, Tk, use, G in reversed(tr["records"]):
        w = a * Tk
        dCda = rgb[:, g][:, None] * Tk[None, :] - S / (1.0 - a)[None, :]
        dLda = np.where(use, (dC * dCda).sum(axis=0), 0.0)
        dLdrgb = np.where(use[None, :], dC * w[None, :], 0.0)
        S = S + np.where(use[None, :], rgb[:, g][:, None] * w[None, :], 0.0)
        unclamped = use & (o[g] * G < I.ALPHA_MAX)
        k = np.where(unclamped, dLda * o[g] * G, 0.0)           # dL/dalpha times alpha
        dx = px - u[g]
        dy = py - v[g]
        A, B, Cc = conic[:, g]
        acc = out.setdefault(int(g), dict(du=0.0, dv=0.0, dA=0.0, dB=0.0, dC=0.0, do=0.0, drgb=np.zeros(3)))
        acc["du"] += float((k * (2.0 * A * dx + 2.0 * B * dy)).sum())
        acc["dv"] += float((k * (2.0 * B * dx + 2.0 * Cc * dy)).sum())
        acc["dA"] += float((-k * dx * dx).sum())
        acc["dB"] += float((-2.0 * k * dx * dy).sum())
        acc["dC"] += float((-k * dy * dy).sum())
        acc["do"] += float((k / o[g]).sum())
        acc["drgb"] = acc["drgb"] + dLdrgb.sum(axis=1)
    return out


_SG_KEYS = ("du", "dv", "dA", "dB", "dC", "do")


def screen_grads_aniso_tiled(u, v, conic, o, rgb, bins, view_id, width, height, dC, bg=(0.0, 0.0, 0.0),
                             pidx_offset=0):
    """Per-particle screen-space gradients of one view over all its tiles. dC is dL/dimage
    [3, H, W]. Returns arrays du, dv, dA, dB, dC, do [n] and drgb [3, n]."""
    n = u.shape[0]
    g = {k: np.zeros(n) for k in _SG_KEYS}
    g["drgb"] = np.zeros((3, n))
    TX, TY = I.tile_grid(width, height)
    base = int(bins.tile_base[view_id])
    for ty in range(TY):
        for tx in range(TX):
            a, b = bins.ranges[base + ty * TX + tx]
            if b <= a:
                continue
            seq = bins.pidx[a:b].astype(np.int64) - pidx_offset
            X, Y = I.tile_pixels(tx, ty, width, height)
            res = composite_backward_aniso(X + 0.5, Y + 0.5, seq, u, v, conic, o, rgb, bg, dC[:, Y, X])
            for gi, acc in res.items():
                for k in _SG_KEYS:
                    g[k][gi] += acc[k]
                g["drgb"][:, gi] += acc["drgb"]
    return g


def _drot_dq(q):
    """d R / d q_j [4][3, 3, n] of quat_to_rot at (not normalised) q [4, n]."""
    w, x, y, z = q
    zero = np.zeros_like(w)
    dw = np.array([[zero, -2 * z, 2 * y], [2 * z, zero, -2 * x], [-2 * y, 2 * x, zero]])
    dx = np.array([[zero, 2 * y, 2 * z], [2 * y, -4 * x, -2 * w], [2 * z, 2 * w, -4 * x]])
    dy = np.array([[-4 * y, 2 * x, 2 * w], [2 * x, zero, 2 * z], [-2 * w, 2 * z, -4 * y]])
    dz = np.array([[-4 * z, -2 * w, 2 * x], [2 * w, -4 * z, 2 * y], [2 * x, 2 * y, zero]])
    return [dw, dx, dy, dz]


def project_backward_aniso64(scene, cam, proj: AnisoProjected64, sg):
    """Chains screen-space gradients to the parameters of one view.

    conic = M^-1 with M = Sigma_2D: with the conic gradient as the symmetric matrix
    Gc = [[dA, dB/2], [dB/2, dC]], dL/dM = -M^-1 Gc M^-1.  M = T Sigma T^T, T = J V:
    dL/dSigma = T^T (dL/dM) T and dL/dT = 2 (dL/dM) T Sigma, dL/dJ = (dL/dT) V^T, and J's
    entries f/z, -f p_x/z^2, -f p_y/z^2 pass their share to p.  Sigma = R diag(s^2) R^T:
    dL/dR = 2 (dL/dSigma) R diag(s^2), dL/ds_i = 2 s_i (R^T (dL/dSigma) R)_ii; R is the
    rotation of q/|q|: dL/dq = (I - qh qh^T)/|q| dL/dqh.  The centre and the colour as in
    the isotropic path (u, v through p; p = V mu + t; the SH direction term).
    Returns dict(pos [3, n], rot [4, n], scale [3, n], opacity [n], color [3K, n]); zero
    for invisible particles. Pinned by finite differences through ``project_aniso64``."""
    V, t, eye, f, cx, cy, near = I._cam64(cam)
    vis = proj.visible
    n = vis.shape[0]
    K = I.sh_count(scene.sh_degree)
    z = np.where(vis, proj.z, 1.0)
    p = np.where(vis[None, :], proj.p, 1.0)
    sc = np.where(vis[None, :], scene.scale.astype(np.float64), 1.0)
    A, B, C = (np.where(vis, x, 0.0) for x in proj.conic)
    Ci = np.array([[A, B], [B, C]])
    Gc = np.array([[sg["dA"], 0.5 * sg["dB"]], [0.5 * sg["dB"], sg["dC"]]])
    Gc = np.where(vis[None, None, :], Gc, 0.0)
    GM = -np.einsum("ikn,kln,ljn->ijn", Ci, Gc, Ci)
    rotm = np.where(vis[None, None, :], proj.rotm, 0.0)
    Sig = covariance3d(rotm, sc)
    J = screen_jacobian(p, f)
    T = np.einsum("ikn,kj->ijn", J, V)
    GSig = np.einsum("kin,kln,ljn->ijn", T, GM, T)
    GT = 2.0 * np.einsum("ikn,kln,ljn->ijn", GM, T, Sig)
    GJ = np.einsum("ikn,jk->ijn", GT, V)
    # J = [[f/z, 0, -f p_x/z^2], [0, f/z, -f p_y/z^2]]
    dpx = -GJ[0, 2] * f / (z * z)
    dpy = -GJ[1, 2] * f / (z * z)
    dpz = (-(GJ[0, 0] + GJ[1, 1]) * f / (z * z) + GJ[0, 2] * 2.0 * f * p[0] / z ** 3
           + GJ[1, 2] * 2.0 * f * p[1] / z ** 3)
    du = np.where(vis, sg["du"], 0.0)
    dv = np.where(vis, sg["dv"], 0.0)
    dpx = dpx + du * f / z
    dpy = dpy + dv * f / z
    dpz = dpz - (du * (proj.u - cx) + dv * (proj.v - cy)) / z
    dp = np.where(vis[None, :], np.stack([dpx, dpy, dpz]), 0.0)
    dmu = V.T @ dp
    # Sigma = R diag(s^2) R^T
    s2 = sc * sc
    GR = 2.0 * np.einsum("ikn,kjn->ijn", GSig, rotm * s2[None, :, :])
    RtGR = np.einsum("kin,kln,ljn->ijn", rotm, GSig, rotm)
    dscale = 2.0 * sc * np.array([RtGR[0, 0], RtGR[1, 1], RtGR[2, 2]])
    qn = np.where(vis, proj.qnorm, 1.0)
    qh = np.where(vis[None, :], scene.rot.astype(np.float64) / qn[None, :], 0.0)
    dqh = np.array([(GR * dR).sum(axis=(0, 1)) for dR in _drot_dq(qh)])
    drot = (dqh - qh * (qh * dqh).sum(axis=0)[None, :]) / qn[None, :]
    # colour (as the isotropic path)
    drgb = np.where(vis[None, :] & (proj.rgb_raw > 0.0), sg["drgb"], 0.0)
    dcolor = np.zeros((K, 3, n))
    dcolor[0] = drgb
    if K > 1:
        dirs1 = np.where(vis[None, :], proj.dirs, 1.0)
        basis = I.sh_basis(scene.sh_degree, dirs1)
        gradY = I.sh_basis_grad(scene.sh_degree, dirs1)
        c3 = scene.color.astype(np.float64).reshape(K, 3, n)
        dd = np.zeros((3, n))
        for k in range(1, K):
            dcolor[k] = drgb * basis[k]
            dd += gradY[k] * (c3[k] * drgb).sum(axis=0)[None, :]
        radial = (proj.dirs * dd).sum(axis=0)
        dmu += np.where(vis[None, :], (dd - proj.dirs * radial[None, :]) / np.where(vis, proj.dist, 1.0), 0.0)
    return dict(pos=dmu, rot=np.where(vis[None, :], drot, 0.0), scale=np.where(vis[None, :], dscale, 0.0),
                opacity=np.where(vis, sg["do"], 0.0), color=dcolor.reshape(3 * K, n))


def scene_grads_aniso(scene, cams, dCs, bg=(0.0, 0.0, 0.0)):
    """dL/d(parameters) for L = sum_v <dC_v, C_v>, views summed in order."""
    projs = [project_aniso64(scene, cam) for cam in cams]
    bins = I.bin_sort_ref(f32_views_aniso(projs, cams))
    total = None
    off = 0
    for vi, (pr, cam, dC) in enumerate(zip(projs, cams, dCs)):
        sg = screen_grads_aniso_tiled(pr.u, pr.v, pr.conic, pr.opacity, pr.rgb, bins, vi, cam.width, cam.height,
                                      np.asarray(dC, dtype=np.float64), bg, pidx_offset=off)
        g = project_backward_aniso64(scene, cam, pr, sg)
        total = g if total is None else {k: total[k] + g[k] for k in g}
        off += pr.u.shape[0]
    return total


def decision_signature_aniso(proj: AnisoProjected64, width, height, bg=(0.0, 0.0, 0.0)):
    """Every discrete decision of an untiled render (visibility, order, the alpha threshold
    of every pair, where each pixel stops, clamps) as bytes: renders with equal signatures
    lie on one smooth branch, across which central differences are valid."""
    seq = depth_order_aniso(proj)
    X, Y = np.meshgrid(np.arange(width), np.arange(height))
    _, _, n_last, tr = composite_pixels_aniso(X.ravel() + 0.5, Y.ravel() + 0.5, seq, proj.u, proj.v, proj.conic,
                                              proj.opacity, proj.rgb, bg, trace=True)
    parts = [proj.visible.tobytes(), seq.tobytes(), n_last.tobytes(), (proj.rgb_raw > 0).tobytes()]
    for pos, g, a, Tk, use, G in tr["records"]:
        parts.append(np.int64(pos).tobytes())
        parts.append(use.tobytes())
        parts.append((use & (proj.opacity[g] * G >= I.ALPHA_MAX)).tobytes())
    return b"".join(parts)
