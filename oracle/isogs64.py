"""FP64 CPU oracle for isotropic Gaussian splatting.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never
calls it and shares no code, constants table or helper with it.

What it computes (paper: Gong, Yu, Yue, "Isotropic Gaussian Splatting for Real-Time
Radiance Field Rendering", arXiv 2403.14244):

* the isotropic kernel g(x) = exp(-|x - mu|^2 / sigma^2) of eq. 8 (no factor 1/2),
  evaluated on the image plane with the screen-space scale s = f sigma / z: Section 2
  ("View Dependency") states an isotropic kernel's size depends only on its distance to
  the view point, not on the view orientation, and Table 1 lists "view dependency: no";
* front-to-back alpha compositing C = sum_k c_k alpha_k prod_{j<k} (1 - alpha_j) of
  eq. 4, k = 1 the nearest particle, with alpha_k = min(0.99, o_k g_k);
* the compact support of eq. 2, read per particle as alpha >= 1/255, which fixes a
  per-particle screen radius used to bin particles into 16 x 16 pixel tiles;
* the gradients of the rendered image with respect to every particle parameter, for
  the back-propagation mode of Section 3 ("Optimization"), derived from eq. 4 and eq. 8
  directly (eq. 3 is written for the un-composited kernel sum and is not used).

Everything is FP64 except where a floating-point comparison decides an integer (tile
membership): there both the oracle and the GPU take the decision in FP32, op by op,
on the same FP32 inputs. Every function states what pins it in the tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg

# Method constants (readings of the paper, see the module docstring).
ALPHA_MIN = 1.0 / 255.0      # eq. 2 support: a particle contributes where alpha >= 1/255
ALPHA_MAX = 0.99             # alpha clamp, keeps 1 - alpha >= 0.01
T_MIN = 1e-4                 # a pixel stops after the entry that takes T below this
TILE = 16                    # tile edge in pixels
RADIUS_GROW = 1.0 + 2.0 ** -10
RADIUS_PAD = 2.0 ** -6


# --------------------------------------------------------------------------------------
# Real spherical harmonics (colour as a function of viewing direction).
# --------------------------------------------------------------------------------------

def sh_count(deg: int) -> int:
    return (deg + 1) ** 2


def _sh_lm(k: int):
    l = int(math.isqrt(k))
    return l, k - l * l - l


def _sh_norm(l: int, m: int) -> float:
    am = abs(m)
    return math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - am) / math.factorial(l + am))


def _xy_power(x, y, m):
    """(x + i y)^m as (real, imag)."""
    z = (x + 1j * y) ** m
    return z.real, z.imag


def sh_basis(deg: int, d: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonics Y_k(d), k = l^2 + l + m, for unit d [3, n].

    Written as polynomials in (x, y, z): for m = 0, K_l^0 P_l(z); for m > 0,
    sqrt(2) K_l^m P_l^(m)(z) Re((x+iy)^m); for m < 0, sqrt(2) K_l^|m| P_l^(|m|)(z)
    Im((x+iy)^|m|), where P_l^(m) is the m-th derivative of the Legendre polynomial and
    K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!). No Condon-Shortley phase, so
    Y_{1,-1}, Y_{1,0}, Y_{1,1} are positive multiples of y, z, x.
    Pinned by orthonormality under quadrature and the degree-1 sign convention.
    """
    x, y, z = (np.asarray(d[i], dtype=np.float64) for i in range(3))
    out = np.empty((sh_count(deg),) + x.shape, dtype=np.float64)
    for k in range(sh_count(deg)):
        l, m = _sh_lm(k)
        am = abs(m)
        q = npleg.legval(z, npleg.legder(npleg.Legendre.basis(l).coef, am)) if am else \
            npleg.legval(z, npleg.Legendre.basis(l).coef)
        if m == 0:
            out[k] = _sh_norm(l, 0) * q
        else:
            re, im = _xy_power(x, y, am)
            out[k] = math.sqrt(2.0) * _sh_norm(l, m) * q * (re if m > 0 else im)
    return out


def sh_basis_grad(deg: int, d: np.ndarray) -> np.ndarray:
    """Gradient of each polynomial Y_k of ``sh_basis`` with respect to (x, y, z): [K, 3, n]."""
    x, y, z = (np.asarray(d[i], dtype=np.float64) for i in range(3))
    out = np.zeros((sh_count(deg), 3) + x.shape, dtype=np.float64)
    for k in range(sh_count(deg)):
        l, m = _sh_lm(k)
        am = abs(m)
        c = npleg.legder(npleg.Legendre.basis(l).coef, am) if am else npleg.Legendre.basis(l).coef
        q = npleg.legval(z, c)
        dq = npleg.legval(z, npleg.legder(c, 1)) if len(c) > 1 else np.zeros_like(z)
        if m == 0:
            out[k, 2] = _sh_norm(l, 0) * dq
            continue
        a = math.sqrt(2.0) * _sh_norm(l, m)
        re, im = _xy_power(x, y, am)
        dre, dim = _xy_power(x, y, am - 1)
        # d/dx (x+iy)^m = m (x+iy)^(m-1); d/dy = i m (x+iy)^(m-1)
        if m > 0:
            ax, ay, base = am * dre, -am * dim, re
        else:
            ax, ay, base = am * dim, am * dre, im
        out[k, 0] = a * q * ax
        out[k, 1] = a * q * ay
        out[k, 2] = a * dq * base
    return out


# --------------------------------------------------------------------------------------
# Projection of isotropic particles to circular screen footprints.
# --------------------------------------------------------------------------------------

@dataclass
class Projected64:
    """FP64 screen footprints of one view (arrays over the scene's particles)."""
    u: np.ndarray
    v: np.ndarray
    z: np.ndarray
    s: np.ndarray          # screen-space scale f sigma / z (pixels)
    opacity: np.ndarray
    rgb: np.ndarray        # [3, n], clamped at 0
    radius: np.ndarray     # binning radius (pixels); 0 where not visible
    visible: np.ndarray    # bool
    # intermediate values kept for the backward pass
    p: np.ndarray          # camera-space position [3, n]
    dirs: np.ndarray       # unit view direction (mu - eye)/|mu - eye| [3, n]
    dist: np.ndarray       # |mu - eye|
    rgb_raw: np.ndarray    # [3, n] before the clamp at 0

    @property
    def inv_s2(self):
        with np.errstate(divide="ignore"):
            return 1.0 / (self.s * self.s)


def _cam64(cam):
    return (np.asarray(cam.R, dtype=np.float64), np.asarray(cam.t, dtype=np.float64),
            np.asarray(cam.eye, dtype=np.float64), float(cam.f), float(cam.cx), float(cam.cy),
            float(cam.near))


def project64(scene, cam) -> Projected64:
    """Footprint of every particle in one view, in FP64 from the FP32 inputs.

    p = R mu + t (world to camera), z = p_z; u = f p_x / z + cx, v = f p_y / z + cy;
    screen scale s = f sigma / z (isotropic footprint, Section 2 "View Dependency");
    rgb = max(0, c_0 + sum_{l>=1} c_lm Y_lm(d)), d = (mu - eye)/|mu - eye|.
    A particle is invisible when any input is non-finite, sigma <= 0, o < 1/255 (it can
    never reach alpha >= 1/255), z <= near, or its footprint has no normal FP32 form (the
    centre, 1/s^2 or the binning radius overflows, or 1/s^2 falls below the smallest normal
    FP32 value).
    Binning radius r = s sqrt(ln(255 o)) (1 + 2^-10) + 2^-6: alpha = o exp(-d^2/s^2) >= 1/255
    exactly when d <= s sqrt(ln(255 o)); the small growth makes the FP32 tile test a
    superset of that disk.
    Pinned by the single-particle closed forms (peak, e^-1 falloff, distance scaling,
    roll invariance) in the oracle tests.
    """
    R, t, eye, f, cx, cy, near = _cam64(cam)
    mu = scene.pos.astype(np.float64)
    sigma = scene.scale.astype(np.float64)
    o = scene.opacity.astype(np.float64)
    coef = scene.color.astype(np.float64)
    n = sigma.shape[0]
    K = sh_count(scene.sh_degree)

    with np.errstate(all="ignore"):
        p = R @ mu + t[:, None]
        z = p[2]
        u = f * p[0] / z + cx
        v = f * p[1] / z + cy
        s = f * sigma / z
        dvec = mu - eye[:, None]
        dist = np.sqrt((dvec * dvec).sum(axis=0))
        dirs = dvec / dist
        basis = sh_basis(scene.sh_degree, dirs)                      # [K, n]
        c3 = coef.reshape(K, 3, n)
        rgb_raw = c3[0].copy()
        for k in range(1, K):
            rgb_raw = rgb_raw + c3[k] * basis[k]
        rgb = np.maximum(rgb_raw, 0.0)
        finite = (np.isfinite(mu).all(axis=0) & np.isfinite(sigma) & np.isfinite(o)
                  & np.isfinite(coef).all(axis=0))
        visible = finite & (sigma > 0) & (o >= ALPHA_MIN) & (z > near)
        visible &= np.isfinite(u) & np.isfinite(v) & np.isfinite(s) & (s > 0) & np.isfinite(rgb).all(axis=0)
        radius = np.where(visible, s * np.sqrt(np.log(np.where(visible, 255.0 * o, 1.0)))
                          * RADIUS_GROW + RADIUS_PAD, 0.0)
        # a footprint must be representable in FP32 (the stored form of every footprint):
        # 1/s^2 finite and at least the smallest normal FP32 value, the binning radius
        # finite, else it is culled
        inv32 = np.where(visible, 1.0 / np.where(visible, s * s, 1.0), 1.0).astype(np.float32)
        visible &= (np.isfinite(inv32) & (inv32 >= np.finfo(np.float32).tiny)
                    & np.isfinite(radius.astype(np.float32)) & np.isfinite(u.astype(np.float32))
                    & np.isfinite(v.astype(np.float32)))
        radius = np.where(visible, radius, 0.0)
    return Projected64(u=u, v=v, z=z, s=s, opacity=o, rgb=rgb, radius=radius, visible=visible,
                       p=p, dirs=dirs, dist=dist, rgb_raw=rgb_raw)


# --------------------------------------------------------------------------------------
# Binning into 16x16 tiles and the depth sort.
# --------------------------------------------------------------------------------------

def tile_grid(width: int, height: int):
    return -(-width // TILE), -(-height // TILE)


def tile_member_f32(u, v, r, tx, ty, width, height):
    """Exact disk-versus-tile test in FP32, one IEEE operation at a time (no fused ops).

    The tile's pixel centres span [16tx + 1/2, min(16tx + 15.5, W - 1/2)] in x (likewise
    in y). dx = max(max(x_lo - u, u - x_hi), 0), dy likewise; member iff
    dx*dx + dy*dy <= r*r. All operands are FP32 arrays; numpy evaluates each operation
    in FP32 with round-to-nearest-even, which is the decision the GPU takes.
    """
    f32 = np.float32
    u, v, r = (np.asarray(a, dtype=f32) for a in (u, v, r))
    tx = np.asarray(tx, dtype=np.int64)
    ty = np.asarray(ty, dtype=np.int64)
    x_lo = (tx * TILE).astype(f32) + f32(0.5)
    y_lo = (ty * TILE).astype(f32) + f32(0.5)
    x_hi = np.minimum((tx * TILE).astype(f32) + f32(15.5), f32(width) - f32(0.5))
    y_hi = np.minimum((ty * TILE).astype(f32) + f32(15.5), f32(height) - f32(0.5))
    dx = np.maximum(np.maximum(x_lo - u, u - x_hi), f32(0.0))
    dy = np.maximum(np.maximum(y_lo - v, v - y_hi), f32(0.0))
    d2 = dx * dx + dy * dy
    return d2 <= r * r


def member_tiles(u, v, r, width, height, brute_force=False):
    """Member tiles of every footprint, in emit order: by particle, then row-major (ty, tx).

    Candidates are the tiles of the footprint's bounding box grown by one tile on every
    side (clipped to the image), or every tile when ``brute_force``; membership is
    ``tile_member_f32``. A particle with r <= 0 or non-finite u, v, r has no tiles.
    Returns (particle index, ty, tx) arrays. Pinned: bounding-box candidates give the
    same lists as brute force; every pixel centre within the FP64 support disk lies in a
    member tile.
    """
    TX, TY = tile_grid(width, height)
    u = np.asarray(u, dtype=np.float32)
    v = np.asarray(v, dtype=np.float32)
    r = np.asarray(r, dtype=np.float32)
    n = u.shape[0]
    ok = np.isfinite(u) & np.isfinite(v) & np.isfinite(r) & (r > 0)
    if brute_force:
        gi, ty, tx = np.meshgrid(np.arange(n), np.arange(TY), np.arange(TX), indexing="ij")
        gi, ty, tx = gi.ravel(), ty.ravel(), tx.ravel()
    else:
        u64, v64, r64 = u.astype(np.float64), v.astype(np.float64), r.astype(np.float64)
        with np.errstate(invalid="ignore"):
            tx0 = np.clip(np.floor((u64 - r64) / TILE) - 1, 0, TX - 1)
            tx1 = np.clip(np.floor((u64 + r64) / TILE) + 1, -1, TX - 1)
            ty0 = np.clip(np.floor((v64 - r64) / TILE) - 1, 0, TY - 1)
            ty1 = np.clip(np.floor((v64 + r64) / TILE) + 1, -1, TY - 1)
        nx = np.where(ok, np.maximum(tx1 - tx0 + 1, 0), 0).astype(np.int64)
        ny = np.where(ok, np.maximum(ty1 - ty0 + 1, 0), 0).astype(np.int64)
        cnt = nx * ny
        gi = np.repeat(np.arange(n), cnt)
        start = np.cumsum(cnt) - cnt
        j = np.arange(gi.shape[0]) - np.repeat(start, cnt)
        nxr = np.repeat(nx, cnt)
        ty = np.repeat(ty0.astype(np.int64), cnt) + j // np.maximum(nxr, 1)
        tx = np.repeat(tx0.astype(np.int64), cnt) + j % np.maximum(nxr, 1)
    keep = ok[gi] & tile_member_f32(u[gi], v[gi], r[gi], tx, ty, width, height)
    return gi[keep], ty[keep], tx[keep]


@dataclass
class Bins:
    keys: np.ndarray        # uint64 [count], sorted ascending
    emit_index: np.ndarray  # uint32 [count]: position of each sorted entry in emit order
    pidx: np.ndarray        # uint32 [count]: particle index (into the packed views) per entry
    ranges: np.ndarray      # uint32 [total_tiles, 2]: [start, end) per tile, empty = [0, 0)
    tile_count: np.ndarray  # uint32 [n_total]: member tiles per particle
    offsets: np.ndarray     # uint32 [n_total]: first emit position per particle
    tile_base: np.ndarray   # int64 [V]: first global tile id of each view


def bin_sort_ref(views):
    """Bins and depth-sorts the footprints of a batch of views.

    ``views`` is a list of dicts with FP32 arrays u, v, z, r (one entry per particle) and
    width, height. Particles of all views are numbered consecutively (view 0 first).
    Global tile id = tile_base[view] + ty * TX + tx, views' tile ranges consecutive.
    Emit order: view, particle, then row-major tile. Each entry's key is
    (global tile id << 32) | bits(z as FP32) (z > 0, so the bit pattern orders like the
    value); entries are sorted stably by key, so equal depths keep emit order. Tile
    ranges are [start, end) into the sorted entries, [0, 0) for an empty tile.
    Pinned against Python's ``sorted`` and a cumulative-sum check in the tests.
    """
    keys, pidx_all, counts_all = [], [], []
    base, n_base = 0, 0
    tile_base = []
    for vw in views:
        W, H = int(vw["width"]), int(vw["height"])
        TX, TY = tile_grid(W, H)
        u, v, z, r = (np.asarray(vw[k], dtype=np.float32) for k in ("u", "v", "z", "r"))
        gi, ty, tx = member_tiles(u, v, r, W, H)
        tid = (base + ty * TX + tx).astype(np.uint64)
        zb = z.view(np.uint32)[gi].astype(np.uint64)
        keys.append((tid << np.uint64(32)) | zb)
        pidx_all.append((gi + n_base).astype(np.uint32))
        counts_all.append(np.bincount(gi, minlength=u.shape[0]).astype(np.uint32))
        tile_base.append(base)
        base += TX * TY
        n_base += u.shape[0]
    keys = np.concatenate(keys) if keys else np.zeros(0, np.uint64)
    pidx = np.concatenate(pidx_all) if pidx_all else np.zeros(0, np.uint32)
    tile_count = np.concatenate(counts_all) if counts_all else np.zeros(0, np.uint32)
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    ranges = np.zeros((base, 2), dtype=np.uint32)
    if skeys.shape[0]:
        tiles = (skeys >> np.uint64(32)).astype(np.int64)
        first = np.ones(tiles.shape[0], bool)
        first[1:] = tiles[1:] != tiles[:-1]
        last = np.ones(tiles.shape[0], bool)
        last[:-1] = tiles[1:] != tiles[:-1]
        idx = np.arange(tiles.shape[0], dtype=np.uint32)
        ranges[tiles[first], 0] = idx[first]
        ranges[tiles[last], 1] = idx[last] + 1
    offsets = (np.cumsum(tile_count, dtype=np.uint64) - tile_count).astype(np.uint32)
    return Bins(keys=skeys, emit_index=order.astype(np.uint32), pidx=pidx[order], ranges=ranges,
                tile_count=tile_count, offsets=offsets, tile_base=np.asarray(tile_base, np.int64))


# --------------------------------------------------------------------------------------
# Compositing (eq. 4) with the isotropic kernel (eq. 8).
# --------------------------------------------------------------------------------------

def composite_pixels(px, py, seq, u, v, s, o, rgb, bg, trace=False, alpha_band=None, term_band=None,
                     pos_err=None, z32=None):
    """Front-to-back compositing of one particle sequence at a set of pixel centres.

    For every pixel (px, py) independently, walking ``seq`` (particle indices in depth
    order): d^2 = (px-u)^2 + (py-v)^2; G = exp(-d^2/s^2) (eq. 8); alpha = min(0.99, o G);
    the entry is skipped when alpha < 1/255; otherwise C += c alpha T (eq. 4), then
    T *= 1 - alpha, and the pixel stops when T < 1e-4. Finally C += T bg.
    Returns (C [3, P], T_final [P], n_last [P]) where n_last is 1 + the sequence position
    of the last contributing entry (0 if none). With ``trace`` it also returns, per
    pixel, the list of (position, alpha, T before) of contributing entries and the
    decision margins used for flagging: a pixel is near a decision when some entry's
    alpha lies within a relative ``alpha_band`` of 1/255, or some T after an entry lies
    within a relative ``term_band`` of 1e-4.

    When the footprints an implementation composites are themselves roundings of these
    ones (an end-to-end comparison), ``pos_err`` [n] bounds each particle's footprint
    centre error in pixels and ``z32`` [n] gives the FP32 depths that order the lists. An
    entry's alpha band then grows by the relative change of exp(-d^2/s^2) that a shift of
    the centre by pos_err in x and y can cause, (2 (|dx| + |dy|) e + 2 e^2) / s^2; the
    band of T grows by what those alpha changes do to T, the sum over the composited
    entries of alpha/(1 - alpha) times that growth; and a pixel is also near a decision
    when two consecutive composited entries have FP32 depths at most one ulp apart (their
    order may differ). Without them the flags are as described above.
    """
    alpha_band = ALPHA_FLAG_REL if alpha_band is None else alpha_band
    term_band = TERM_FLAG_REL if term_band is None else term_band
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
        d2 = dx * dx + dy * dy
        G = np.exp(-d2 / (s[g] * s[g]))
        a = np.minimum(ALPHA_MAX, o[g] * G)
        live = ~done
        grow = 0.0
        if pos_err is not None:
            e = float(pos_err[g])
            grow = (2.0 * (np.abs(dx) + np.abs(dy)) * e + 2.0 * e * e) / (s[g] * s[g])
        near_alpha |= live & (np.abs(a * 255.0 - 1.0) <= alpha_band + grow)
        use = live & (a >= ALPHA_MIN)
        if not use.any():
            continue
        w = np.where(use, a * T, 0.0)
        C = C + rgb[:, g][:, None] * w[None, :]
        T_new = np.where(use, T * (1.0 - a), T)
        if pos_err is not None:
            t_band = t_band + np.where(use, a / (1.0 - a) * grow, 0.0)
        near_term |= use & (np.abs(T_new / T_MIN - 1.0) <= t_band)
        if zb is not None:
            near_alpha |= use & (np.abs(zb[g] - prev_z) <= 1)
            prev_z = np.where(use, zb[g], prev_z)
        if trace:
            rec.append((pos, g, np.where(use, a, 0.0), T.copy(), use.copy(), G))
        T = T_new
        n_last = np.where(use, pos + 1, n_last)
        done |= use & (T < T_MIN)
    C = C + T[None, :] * np.asarray(bg, dtype=np.float64)[:, None]
    if trace:
        return C, T, n_last, dict(records=rec, near_alpha=near_alpha, near_term=near_term)
    return C, T, n_last


# Relative width of the decision bands inside which FP32 and FP64 may legitimately take
# different discrete decisions (alpha threshold, termination). Pixels whose sequence
# passes through such a band are flagged and compared against a looser bound.
ALPHA_FLAG_REL = 2.0 ** -14
TERM_FLAG_REL = 2.0 ** -10


def pixel_outcomes(px, py, seq, u, v, s, o, rgb, bg=(0.0, 0.0, 0.0), alpha_band=None, term_band=None,
                   pos_err=None, z32=None, slack=1e-5, max_branch=12):
    """Every result one pixel can validly take when an FP32 walk and this FP64 walk may
    take a discrete decision differently ("several results are correct").

    The walk of eq. 4 decides, per entry, whether alpha >= 1/255 (the compact support of
    eq. 2) and whether T has fallen below 1e-4 (stop after this entry). When the FP64
    value of such a decision lies within its band of the threshold (the bands and their
    growth with ``pos_err`` as in ``composite_pixels``), an FP32 implementation may take
    either side, and both results are correct. With ``z32``, two consecutive entries that
    may composite and whose FP32 depths are at most one ulp apart may also be taken in
    either order.

    Entries after the first one where even the largest possible T (every in-band entry
    skipped) is clearly below 1e-4 cannot be composited on any branch and are not taken
    both ways. Each remaining alpha decision and order is taken both ways, except alpha
    decisions whose largest possible effect on the colour, 2 M (1/255)(1 + band) T_max (T_max: the
    transmittance before the entry with every in-band entry left out, M the largest
    colour or background magnitude), summed over the decisions left out, stays below
    ``slack``: those keep the FP64 side, and the change of T they could cause widens the
    band of every later stop decision. Along each combination the stop decisions are
    taken both ways inside the band: the walk may stop at every in-band entry up to the
    first entry whose T is clearly below 1e-4, where it must stop (or run to the end of
    the list).

    Returns (outcomes, resolved): outcomes is a list of (C [3], T_final, n_last) with
    n_last the 1-based position of the last composited entry in the (possibly reordered)
    list; resolved is False, with no outcomes, when more than ``max_branch`` decisions
    would have to be taken both ways. Pinned by closed forms of eq. 4 for pixels with one
    in-band alpha, T or order decision, and by agreement with ``composite_pixels`` where
    nothing is in band.
    """
    seq = np.asarray(seq, dtype=np.int64)
    n = seq.shape[0]
    if n == 0:
        return [(np.asarray(bg, dtype=np.float64).copy(), 1.0, 0)], True
    dx = float(px) - u[seq]
    dy = float(py) - v[seq]
    d2 = dx * dx + dy * dy
    s2 = s[seq] * s[seq]
    a = np.minimum(ALPHA_MAX, o[seq] * np.exp(-d2 / s2))
    grow = np.zeros(n)
    if pos_err is not None:
        e = np.asarray(pos_err, dtype=np.float64)[seq]
        grow = (2.0 * (np.abs(dx) + np.abs(dy)) * e + 2.0 * e * e) / s2
    zs = None if z32 is None else np.asarray(z32, dtype=np.float32)[seq]
    return walk_outcomes(a, grow, rgb[:, seq], bg, alpha_band, term_band, zs, slack, max_branch)


def walk_outcomes(a, grow, rgb_seq, bg=(0.0, 0.0, 0.0), alpha_band=None, term_band=None, z32_seq=None, slack=1e-5,
                  max_branch=12):
    """The valid results of one pixel's walk (see ``pixel_outcomes``) from the alpha of each
    entry of its list in list order (clamped, before the 1/255 test), the growth of each
    entry's alpha band, the entries' colours [3, n] and, optionally, their FP32 depths.
    Shared by the kernels whose alpha is computed differently (isotropic, anisotropic)."""
    alpha_band = ALPHA_FLAG_REL if alpha_band is None else alpha_band
    term_band = TERM_FLAG_REL if term_band is None else term_band
    bgv = np.asarray(bg, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    grow = np.asarray(grow, dtype=np.float64)
    n = a.shape[0]
    if n == 0:
        return [(bgv.copy(), 1.0, 0)], True
    ok = a >= ALPHA_MIN
    in_band = np.abs(a * 255.0 - 1.0) <= alpha_band + grow
    # transmittance before each entry, largest over every branch: in-band entries left out
    kept = np.where(ok & ~in_band, 1.0 - a, 1.0)
    T_max_after = np.cumprod(kept)
    T_max = np.concatenate([[1.0], T_max_after[:-1]])
    # every branch has stopped by the first entry whose largest T is clearly below 1e-4
    # (the widest stop band any branch can have): later entries cannot matter
    ratio = a / (1.0 - a)
    widest = term_band + float(np.sum(np.where(ok | in_band, ratio * grow, 0.0))) + float(
        np.sum(np.where(in_band, ratio, 0.0)))
    below = np.nonzero(T_max_after < T_MIN * (1.0 - widest))[0]
    if below.size:
        in_band[below[0] + 1:] = False
    M = max(1.0, float(np.abs(rgb_seq).max()), float(np.abs(bgv).max()))
    effect = 2.0 * M * (1.0 / 255.0) * (1.0 + alpha_band + grow) * T_max
    cand = np.nonzero(in_band)[0]
    cand = cand[np.argsort(-effect[cand], kind="stable")]
    left = float(effect[cand].sum())
    branch = []
    for k in cand:
        if left <= slack:
            break
        branch.append(int(k))
        left -= float(effect[k])
    fixed = np.zeros(n, dtype=bool)
    fixed[cand] = True
    fixed[branch] = False          # in-band decisions kept on the FP64 side
    swaps = []
    if z32_seq is not None:
        zb = np.asarray(z32_seq, dtype=np.float32).view(np.int32).astype(np.int64)
        maybe = np.nonzero(ok | in_band)[0]
        if below.size:
            maybe = maybe[maybe <= below[0]]
        for i0, i1 in zip(maybe[:-1], maybe[1:]):
            if abs(int(zb[i1]) - int(zb[i0])) <= 1:
                swaps.append((int(i0), int(i1)))
    if len(branch) + len(swaps) > max_branch:
        return [], False
    ratio_a = ratio
    outcomes = []
    seen = set()
    nb = len(branch)
    for bits in range(1 << (nb + len(swaps))):
        inc = ok.copy()
        for j, k in enumerate(branch):
            if (bits >> j) & 1:
                inc[k] = not ok[k]
        perm = np.arange(n)
        for j, (i0, i1) in enumerate(swaps):
            if (bits >> (nb + j)) & 1:
                perm[i0], perm[i1] = perm[i1], perm[i0]
        ap, incp = a[perm], inc[perm]
        f = np.where(incp, 1.0 - ap, 1.0)
        T_after = np.cumprod(f)
        T_before = np.concatenate([[1.0], T_after[:-1]])
        w = np.where(incp, ap * T_before, 0.0)
        C_cum = np.cumsum(rgb_seq[:, perm] * w[None, :], axis=1)
        # band of each stop decision: rounding band, plus what the alpha uncertainty of the
        # composited entries and the flips kept on the FP64 side can do to T
        t_band = (term_band + np.cumsum(np.where(incp, ratio_a[perm] * grow[perm], 0.0))
                  + np.cumsum(np.where(fixed[perm], ratio_a[perm], 0.0)))
        stops = []
        for k in np.nonzero(incp)[0]:
            r = T_after[k] / T_MIN
            if abs(r - 1.0) <= t_band[k]:
                stops.append(int(k))
            elif r < 1.0:
                stops.append(int(k))
                break
        else:
            stops.append(-1)       # runs to the end of the list
        for k in stops:
            if k < 0:
                used = np.nonzero(incp)[0]
                Cf = C_cum[:, -1] + T_after[-1] * bgv
                out = (Cf, float(T_after[-1]), int(used[-1]) + 1 if used.size else 0)
            else:
                out = (C_cum[:, k] + T_after[k] * bgv, float(T_after[k]), k + 1)
            key = tuple(np.round(out[0], 12)) + (round(out[1], 12), out[2])
            if key not in seen:
                seen.add(key)
                outcomes.append(out)
    return outcomes, True


def footprint_uncertainty(proj: Projected64):
    """Bounds for comparing against footprints that are the FP32 roundings of these values
    (computed in higher precision and rounded once): each particle's centre error, half an
    FP32 ulp of its larger coordinate (the ulp taken just above the value, so that a
    rounding up into the next binade is covered), and the oracle's FP32 depths (whose
    order an implementation shares up to one ulp). For ``composite_pixels`` and
    ``pixel_outcomes``."""
    grow = 1.0 + 2.0 ** -10
    u32 = (np.abs(np.where(proj.visible, proj.u, 0.0)) * grow).astype(np.float32)
    v32 = (np.abs(np.where(proj.visible, proj.v, 0.0)) * grow).astype(np.float32)
    ulp = np.maximum(np.spacing(u32), np.spacing(v32)).astype(np.float64)
    z32 = np.where(proj.visible, proj.z, 1.0).astype(np.float32)
    return 0.5 * ulp, z32


def depth_order(proj: Projected64):
    """Visible particles in compositing order: ascending depth, ties by index (eq. 4
    indexes particles from the nearest)."""
    idx = np.nonzero(proj.visible)[0]
    return idx[np.lexsort((idx, proj.z[idx]))]


def render64_untiled(proj: Projected64, width, height, bg=(0.0, 0.0, 0.0), rows=None):
    """The plain definition: every pixel walks every visible particle in depth order.

    Returns image [3, H, W] and T_final [H, W]. ``rows``
    optionally restricts the work to a list of pixel rows (others are left zero).
    """
    seq = depth_order(proj)
    img = np.zeros((3, height, width))
    Tf = np.zeros((height, width))
    rows = np.arange(height) if rows is None else np.asarray(rows)
    band = max(1, 65536 // max(width, 1))
    for c0 in range(0, rows.shape[0], band):
        rr = rows[c0:c0 + band]
        X, Y = np.meshgrid(np.arange(width), rr)
        C, T, _ = composite_pixels(X.ravel() + 0.5, Y.ravel() + 0.5, seq, proj.u, proj.v, proj.s,
                                   proj.opacity, proj.rgb, bg)
        img[:, Y.ravel(), X.ravel()] = C
        Tf[Y.ravel(), X.ravel()] = T
    return img, Tf


def tile_pixels(tx, ty, width, height):
    xs = np.arange(tx * TILE, min(tx * TILE + TILE, width))
    ys = np.arange(ty * TILE, min(ty * TILE + TILE, height))
    X, Y = np.meshgrid(xs, ys)
    return X.ravel(), Y.ravel()


def render64_tiled(u, v, s, o, rgb, bins: Bins, view_id, width, height, bg=(0.0, 0.0, 0.0),
                   tiles=None, pidx_offset=0, with_flags=False, alpha_band=None, term_band=None,
                   pos_err=None, z32=None):
    """Per-tile rendering of one view: each pixel walks its tile's sorted entry list.

    u, v, s, o, rgb are per-particle arrays of this view (upcast to FP64); ``bins`` comes
    from ``bin_sort_ref``; entry particle indices are relative to ``pidx_offset``.
    Returns image [3, H, W], T_final [H, W], n_last [H, W] (positions in the tile list),
    and with ``with_flags`` the near-decision flag mask. ``tiles`` optionally restricts the
    work to a list of (tx, ty). Pinned: bitwise equal to ``render64_untiled`` in FP64.
    """
    TX, TY = tile_grid(width, height)
    img = np.zeros((3, height, width))
    Tf = np.ones((height, width))
    nl = np.zeros((height, width), dtype=np.int64)
    flags = np.zeros((height, width), dtype=bool)
    tiles = [(tx, ty) for ty in range(TY) for tx in range(TX)] if tiles is None else tiles
    base = int(bins.tile_base[view_id])
    for tx, ty in tiles:
        a, b = bins.ranges[base + ty * TX + tx]
        seq = bins.pidx[a:b].astype(np.int64) - pidx_offset
        X, Y = tile_pixels(tx, ty, width, height)
        C, T, n, tr = composite_pixels(X + 0.5, Y + 0.5, seq, u, v, s, o, rgb, bg, trace=True,
                                       alpha_band=alpha_band, term_band=term_band, pos_err=pos_err, z32=z32)
        img[:, Y, X] = C
        Tf[Y, X] = T
        nl[Y, X] = n
        flags[Y, X] = tr["near_alpha"] | tr["near_term"]
    if with_flags:
        return img, Tf, nl, flags
    return img, Tf, nl


# --------------------------------------------------------------------------------------
# Backward: gradients of the rendered image for back-propagation.
# --------------------------------------------------------------------------------------

def composite_backward_pixels(px, py, seq, u, v, s, o, rgb, bg, dC):
    """Gradient of L = sum_p <dC[:, p], C_p> with respect to each sequence entry's
    screen parameters, from eq. 4 and eq. 8.

    With T_k the transmittance before entry k and S_k = sum_{j>k} c_j alpha_j T_j
    + T_final bg (the light arriving from behind k):
      dC/dc_k = alpha_k T_k;   dC/dalpha_k = c_k T_k - S_k / (1 - alpha_k);
      alpha = min(0.99, o G): dalpha/do = G and dalpha/dG = o when o G < 0.99, else 0;
      G = exp(-d^2/s^2): dG/du = 2 G (x-u)/s^2, dG/dv = 2 G (y-v)/s^2, dG/ds = 2 G d^2/s^3.
    Skipped entries and the discrete decisions (threshold, termination, order) carry no
    gradient. Returns a dict of per-particle sums over the pixels: du, dv, ds, do, drgb.
    Pinned by central finite differences of ``composite_pixels``.
    """
    C, T, n_last, tr = composite_pixels(px, py, seq, u, v, s, o, rgb, bg, trace=True)
    P = px.shape[0]
    S = T[None, :] * np.asarray(bg, dtype=np.float64)[:, None]       # [3, P]
    out = {}
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    for pos, g, a, Tk, use, G in reversed(tr["records"]):
        w = a * Tk                                                    # alpha T
        dCda = rgb[:, g][:, None] * Tk[None, :] - S / (1.0 - a)[None, :]
        dLda = np.where(use, (dC * dCda).sum(axis=0), 0.0)
        dLdrgb = np.where(use[None, :], dC * w[None, :], 0.0)
        S = S + np.where(use[None, :], rgb[:, g][:, None] * w[None, :], 0.0)
        unclamped = use & (o[g] * G < ALPHA_MAX)
        dLdG = np.where(unclamped, dLda * o[g], 0.0)
        dLdo = np.where(unclamped, dLda * G, 0.0)
        dx = px - u[g]
        dy = py - v[g]
        d2 = dx * dx + dy * dy
        s2 = s[g] * s[g]
        acc = out.setdefault(int(g), dict(du=0.0, dv=0.0, ds=0.0, do=0.0, drgb=np.zeros(3)))
        acc["du"] += float((dLdG * 2.0 * G * dx / s2).sum())
        acc["dv"] += float((dLdG * 2.0 * G * dy / s2).sum())
        acc["ds"] += float((dLdG * 2.0 * G * d2 / (s2 * s[g])).sum())
        acc["do"] += float(dLdo.sum())
        acc["drgb"] = acc["drgb"] + dLdrgb.sum(axis=1)
    return out


def screen_grads_tiled(u, v, s, o, rgb, bins: Bins, view_id, width, height, dC, bg=(0.0, 0.0, 0.0),
                       pidx_offset=0):
    """Per-particle screen-space gradients of one view, summed over all its tiles.
    dC is dL/dimage [3, H, W]. Returns arrays du, dv, ds, do [n] and drgb [3, n]."""
    n = u.shape[0]
    g = dict(du=np.zeros(n), dv=np.zeros(n), ds=np.zeros(n), do=np.zeros(n), drgb=np.zeros((3, n)))
    TX, TY = tile_grid(width, height)
    base = int(bins.tile_base[view_id])
    for ty in range(TY):
        for tx in range(TX):
            a, b = bins.ranges[base + ty * TX + tx]
            if b <= a:
                continue
            seq = bins.pidx[a:b].astype(np.int64) - pidx_offset
            X, Y = tile_pixels(tx, ty, width, height)
            res = composite_backward_pixels(X + 0.5, Y + 0.5, seq, u, v, s, o, rgb, bg, dC[:, Y, X])
            for gi, acc in res.items():
                g["du"][gi] += acc["du"]
                g["dv"][gi] += acc["dv"]
                g["ds"][gi] += acc["ds"]
                g["do"][gi] += acc["do"]
                g["drgb"][:, gi] += acc["drgb"]
    return g


def screen_grads_untiled(proj: Projected64, width, height, dC, bg=(0.0, 0.0, 0.0)):
    """As ``screen_grads_tiled`` but every pixel walks every visible particle."""
    n = proj.u.shape[0]
    g = dict(du=np.zeros(n), dv=np.zeros(n), ds=np.zeros(n), do=np.zeros(n), drgb=np.zeros((3, n)))
    seq = depth_order(proj)
    X, Y = np.meshgrid(np.arange(width), np.arange(height))
    X, Y = X.ravel(), Y.ravel()
    for c0 in range(0, X.shape[0], 65536):
        xs, ys = X[c0:c0 + 65536], Y[c0:c0 + 65536]
        res = composite_backward_pixels(xs + 0.5, ys + 0.5, seq, proj.u, proj.v, proj.s,
                                        proj.opacity, proj.rgb, bg, dC[:, ys, xs])
        for gi, acc in res.items():
            g["du"][gi] += acc["du"]
            g["dv"][gi] += acc["dv"]
            g["ds"][gi] += acc["ds"]
            g["do"][gi] += acc["do"]
            g["drgb"][:, gi] += acc["drgb"]
    return g


def project_backward64(scene, cam, proj: Projected64, sg):
    """Chains screen-space gradients to the scene parameters of one view.

    s = f sigma / z:  dL/dsigma = dL/ds f/z;  the depth receives -dL/ds s/z.
    u = f p_x/z + cx, v = f p_y/z + cy:  dL/dp_x = dL/du f/z, dL/dp_y = dL/dv f/z,
      dL/dp_z -= (dL/du (u - cx) + dL/dv (v - cy)) / z.
    p = R mu + t:  dL/dmu = R^T dL/dp.
    rgb = max(0, c_0 + sum_k c_k Y_k(d)), d = (mu - eye)/|mu - eye|, where the value
      before the clamp is positive: dL/dc_0 = dL/drgb, dL/dc_k = dL/drgb Y_k(d), and
      dL/dmu += (I - d d^T)/|mu - eye| sum_k c_k grad Y_k(d) dL/drgb.
    Invisible particles get zero. Returns dict(pos [3,n], scale [n], opacity [n],
    color [3K, n]). Pinned by finite differences through ``project64``.
    """
    R, t, eye, f, cx, cy, near = _cam64(cam)
    vis = proj.visible
    z = np.where(vis, proj.z, 1.0)
    sigma = scene.scale.astype(np.float64)
    n = sigma.shape[0]
    K = sh_count(scene.sh_degree)
    du = np.where(vis, sg["du"], 0.0)
    dv = np.where(vis, sg["dv"], 0.0)
    ds = np.where(vis, sg["ds"], 0.0)
    dsigma = ds * f / z
    dpx = du * f / z
    dpy = dv * f / z
    dpz = -ds * proj.s / z - (du * (proj.u - cx) + dv * (proj.v - cy)) / z
    dp = np.stack([dpx, dpy, np.where(vis, dpz, 0.0)])
    dmu = R.T @ dp
    drgb = np.where(vis[None, :] & (proj.rgb_raw > 0.0), sg["drgb"], 0.0)   # [3, n]
    dcolor = np.zeros((K, 3, n))
    dcolor[0] = drgb
    if K > 1:
        basis = sh_basis(scene.sh_degree, np.where(vis[None, :], proj.dirs, 1.0))
        gradY = sh_basis_grad(scene.sh_degree, np.where(vis[None, :], proj.dirs, 1.0))   # [K,3,n]
        c3 = scene.color.astype(np.float64).reshape(K, 3, n)
        dd = np.zeros((3, n))
        for k in range(1, K):
            dcolor[k] = drgb * basis[k]
            w = (c3[k] * drgb).sum(axis=0)                 # sum over channels of c_k,ch dL/drgb_ch
            dd += gradY[k] * w[None, :]
        dirs = proj.dirs
        radial = (dirs * dd).sum(axis=0)
        dmu += np.where(vis[None, :], (dd - dirs * radial[None, :]) / np.where(vis, proj.dist, 1.0), 0.0)
    return dict(pos=dmu, scale=dsigma, opacity=np.where(vis, sg["do"], 0.0),
                color=dcolor.reshape(3 * K, n))


# --------------------------------------------------------------------------------------
# Whole-pipeline drivers used by the tests and the CPU baseline.
# --------------------------------------------------------------------------------------

def f32_views(projs, cams):
    """The FP32 binning inputs (u, v, z, r) of FP64 footprints, one dict per view.
    Invisible particles get r = 0 (no tiles)."""
    out = []
    for pr, cam in zip(projs, cams):
        r = np.where(pr.visible, pr.radius, 0.0)
        out.append(dict(u=np.where(pr.visible, pr.u, 0.0).astype(np.float32),
                        v=np.where(pr.visible, pr.v, 0.0).astype(np.float32),
                        z=np.where(pr.visible, pr.z, 1.0).astype(np.float32),
                        r=r.astype(np.float32), width=cam.width, height=cam.height))
    return out


def render_views(scenes, cams, bg=(0.0, 0.0, 0.0), tiles=None, alpha_band=None, term_band=None,
                 rounded=False):
    """Projects, bins and renders each (scene, camera) pair with the tiled oracle.

    Footprints are FP64; binning takes its decisions on their FP32 roundings. With
    ``rounded`` the flags also cover what FP32 footprints computed elsewhere may change
    (``footprint_uncertainty``).
    Returns (images list, T_final list, n_last list, flags list, projections, bins)."""
    projs = [project64(sc, cam) for sc, cam in zip(scenes, cams)]
    bins = bin_sort_ref(f32_views(projs, cams))
    imgs, Ts, nls, fls = [], [], [], []
    off = 0
    for vi, (pr, cam) in enumerate(zip(projs, cams)):
        pe, z32 = footprint_uncertainty(pr) if rounded else (None, None)
        img, Tf, nl, fl = render64_tiled(pr.u, pr.v, pr.s, pr.opacity, pr.rgb, bins, vi, cam.width,
                                         cam.height, bg, tiles=tiles, pidx_offset=off, with_flags=True,
                                         alpha_band=alpha_band, term_band=term_band, pos_err=pe, z32=z32)
        imgs.append(img)
        Ts.append(Tf)
        nls.append(nl)
        fls.append(fl)
        off += pr.u.shape[0]
    return imgs, Ts, nls, fls, projs, bins


def scene_grads(scene, cams, dCs, bg=(0.0, 0.0, 0.0)):
    """dL/d(scene parameters) for L = sum_v <dC_v, C_v>, views summed in order."""
    projs = [project64(scene, cam) for cam in cams]
    bins = bin_sort_ref(f32_views(projs, cams))
    total = None
    off = 0
    for vi, (pr, cam, dC) in enumerate(zip(projs, cams, dCs)):
        sg = screen_grads_tiled(pr.u, pr.v, pr.s, pr.opacity, pr.rgb, bins, vi, cam.width, cam.height,
                                np.asarray(dC, dtype=np.float64), bg, pidx_offset=off)
        g = project_backward64(scene, cam, pr, sg)
        total = g if total is None else {k: total[k] + g[k] for k in g}
        off += pr.u.shape[0]
    return total


def decision_signature(proj: Projected64, width, height, bg=(0.0, 0.0, 0.0)):
    """Every discrete decision of an untiled render, as bytes: visibility, depth order,
    which (pixel, entry) pairs pass alpha >= 1/255, where each pixel stops, which alphas
    are clamped at 0.99 and which colour channels are clamped at 0. Two renders with the
    same signature are on the same smooth branch, so central finite differences across
    them are valid (the gradient ignores the decisions themselves)."""
    seq = depth_order(proj)
    X, Y = np.meshgrid(np.arange(width), np.arange(height))
    _, _, n_last, tr = composite_pixels(X.ravel() + 0.5, Y.ravel() + 0.5, seq, proj.u, proj.v,
                                        proj.s, proj.opacity, proj.rgb, bg, trace=True)
    parts = [proj.visible.tobytes(), seq.tobytes(), n_last.tobytes(),
             (proj.rgb_raw > 0).tobytes()]
    for pos, g, a, Tk, use, G in tr["records"]:
        parts.append(np.int64(pos).tobytes())
        parts.append(use.tobytes())
        parts.append((use & (proj.opacity[g] * G >= ALPHA_MAX)).tobytes())
    return b"".join(parts)
