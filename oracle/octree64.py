"""Oracle of the octree initialisation of 3D particles and of the merge of 2D particles (the
paper's Section 3, "Initial with Tree Structure", and Section 2, "Multiscale").

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never calls
it and shares no code, constants table or helper with it.

Octree initialisation. The paper manages 3D particles with an octree, as the 2D ones with
a quadtree: every leaf cell carries a particle with the average colour of its region and a
scale of half the cell width. The 3D signal the tree is built over is, here, a coloured
point cloud (the stand-in for the points a reconstruction starts from). Readings:

* the domain is a grid of cubic root cells of edge `root_side` with corner `lo`,
  roots[0] x roots[1] x roots[2] of them; the tree has `levels` levels, level l having
  cells of edge root_side / 2^l; a point belongs to the finest cell
  floor((p - lo) / h) (FP64, per axis, h the finest edge) and is ignored outside the grid;
* cell statistics are exact integers: each colour channel, clamped to [0, 1], is
  quantised to q = rint(65535 c) (round half to even), and a cell keeps its point count n,
  the sums of q and of q^2 per channel; coarser cells add their eight children. The colour
  variance of a cell, in FP64 from those integers, is
  (1/3) sum_ch (S2_ch / n - (S1_ch / n)^2), compared with tau 65535^2 (tau for colours in
  [0, 1]). Exact sums make the statistics independent of the order points are added in;
* a cell with no point is never split and carries no particle; a non-empty cell of a level
  below the last splits into its (non-empty) octants when its variance exceeds tau;
* the tree grows level by level and the particle budget K is kept by refusing a whole
  level, as for the quadtree: if the leaves so far, plus the non-empty cells of the level
  that do not split, plus the non-empty children of the splitting ones, would exceed K,
  no cell of the level splits;
* leaves are numbered level by level, x fastest, then y, then z within a level; a leaf's
  particle: centre = the cell's centre lo + (i + 1/2) edge (FP64, rounded to FP32), scale =
  edge / 2, opacity = the given initial value, colour = the mean quantised colour / 65535
  (FP64, rounded to FP32), as the degree-0 colour coefficient.

Merge of 2D particles (Section 2: isotropic kernels are easily merged, divided, deleted or
added according to their scale; Section 3, "Optimization": particles can be merged or
split). Reading: the inverse of the quadtree split. Particles with sigma <= sigma_max (and
finite parameters, sigma > 0, centre inside the image) are grouped by the square cell of
edge `cell` containing their centre (floor(mu / cell), FP64); every group of at least two
particles becomes one particle that keeps the kernels' total mass per channel
(the integral of A exp(-|x - mu|^2 / sigma^2) is pi A sigma^2):
  sigma_m^2 = sum sigma_k^2, mu_m = sum sigma_k^2 mu_k / sigma_m^2,
  A_m = sum sigma_k^2 A_k / sigma_m^2,
so the four children of a split merge back into their parent exactly. The merged particle
takes the place of the group's first member (in input order); all other particles keep
their order. Sums in FP64.
"""
from __future__ import annotations

import numpy as np

QMAX = 65535.0


def _quantise(colors):
    c = np.clip(np.asarray(colors, dtype=np.float32).astype(np.float64), 0.0, 1.0)
    return np.rint(c * QMAX).astype(np.int64)


def finest_cells(points, lo, root_side, roots, levels):
    """Finest-cell coordinates [3, P] of every point (-1 where outside the grid)."""
    p = np.asarray(points, dtype=np.float32).astype(np.float64)
    lo64 = np.asarray(lo, dtype=np.float32).astype(np.float64)
    h = float(np.float32(root_side)) / float(1 << (levels - 1))
    dims = np.asarray(roots, dtype=np.int64) << (levels - 1)
    with np.errstate(invalid="ignore"):
        idx = np.floor((p - lo64[:, None]) / h)
    ok = np.isfinite(idx).all(axis=0) & (idx >= 0).all(axis=0) & (idx < dims[:, None]).all(axis=0)
    out = np.where(ok[None, :], idx, -1).astype(np.int64)
    return out, ok


def level_stats(points, colors, lo, root_side, roots, levels):
    """Integer statistics of every level: list of (n [gz, gy, gx], S1 [3, gz, gy, gx],
    S2 [3, ...]), level 0 first."""
    idx, ok = finest_cells(points, lo, root_side, roots, levels)
    q = _quantise(colors)
    gx, gy, gz = (int(r) << (levels - 1) for r in roots)
    n = np.zeros((gz, gy, gx), dtype=np.int64)
    S1 = np.zeros((3, gz, gy, gx), dtype=np.int64)
    S2 = np.zeros((3, gz, gy, gx), dtype=np.int64)
    i, j, k = idx[0][ok], idx[1][ok], idx[2][ok]
    np.add.at(n, (k, j, i), 1)
    for ch in range(3):
        np.add.at(S1[ch], (k, j, i), q[ch][ok])
        np.add.at(S2[ch], (k, j, i), q[ch][ok] * q[ch][ok])
    stats = [(n, S1, S2)]
    for _ in range(levels - 1):
        n, S1, S2 = stats[0]
        up = lambda a: a.reshape(*a.shape[:-3], a.shape[-3] // 2, 2, a.shape[-2] // 2, 2, a.shape[-1] // 2, 2).sum(
            axis=(-5, -3, -1))
        stats.insert(0, (up(n), up(S1), up(S2)))
    return stats


def cell_variance(n, S1, S2):
    """(1/3) sum_ch (S2/n - (S1/n)^2) in FP64 (quantised units), NaN where n = 0."""
    with np.errstate(invalid="ignore", divide="ignore"):
        nd = n.astype(np.float64)
        v = np.zeros(n.shape)
        for ch in range(3):
            m = S1[ch].astype(np.float64) / nd
            v = v + (S2[ch].astype(np.float64) / nd - m * m)
        return v / 3.0


def octree_init64(points, colors, lo, root_side, roots, levels, tau, K, opacity=0.5):
    """Particles of the octree leaves: dict(pos [3, m], scale [m], opacity [m], color [3, m],
    count) with m = min(count, K); count is the number of leaves (it exceeds K only when the
    non-empty root cells alone do)."""
    stats = level_stats(points, colors, lo, root_side, roots, levels)
    thr = float(np.float32(tau)) * QMAX * QMAX
    lo64 = np.asarray(lo, dtype=np.float32).astype(np.float64)
    side0 = float(np.float32(root_side))
    leaves = []           # (level, flat cells of the level)
    done = 0
    active = np.ones(stats[0][0].shape, dtype=bool)
    for l, (n, S1, S2) in enumerate(stats):
        nonempty = n > 0
        has_next = l + 1 < levels
        if has_next:
            split = active & nonempty & (cell_variance(n, S1, S2) > thr)
            nk = stats[l + 1][0] > 0
            kids = nk.reshape(n.shape[0], 2, n.shape[1], 2, n.shape[2], 2).sum(axis=(1, 3, 5))
        else:
            split = np.zeros_like(active)
            kids = np.zeros(n.shape, dtype=np.int64)
        leaf = active & nonempty & ~split
        if done + int(leaf.sum()) + int(kids[split].sum()) > K:
            split[:] = False
            leaf = active & nonempty
        leaves.append((l, np.flatnonzero(leaf.ravel())))
        done += int(leaf.sum())
        if has_next:
            active = np.repeat(np.repeat(np.repeat(split, 2, axis=0), 2, axis=1), 2, axis=2)
    pos, scale, color = [], [], []
    for l, cells in leaves:
        n, S1, _ = stats[l]
        gz, gy, gx = n.shape
        edge = side0 / float(1 << l)
        k, rem = np.divmod(cells, gy * gx)
        j, i = np.divmod(rem, gx)
        centre = lo64[:, None] + (np.stack([i, j, k]).astype(np.float64) + 0.5) * edge
        pos.append(centre)
        scale.append(np.full(cells.shape[0], 0.5 * edge))
        nn = n.ravel()[cells].astype(np.float64)
        color.append(np.stack([S1[ch].ravel()[cells].astype(np.float64) / nn / QMAX for ch in range(3)]))
    pos = np.concatenate(pos, axis=1) if pos else np.zeros((3, 0))
    scale = np.concatenate(scale) if scale else np.zeros(0)
    color = np.concatenate(color, axis=1) if color else np.zeros((3, 0))
    count = pos.shape[1]
    m = min(count, K)
    return dict(pos=pos[:, :m].astype(np.float32), scale=scale[:m].astype(np.float32),
                opacity=np.full(m, np.float32(opacity), np.float32), color=color[:, :m].astype(np.float32),
                count=count)


def octree_init_recursive(points, colors, lo, root_side, roots, levels, tau):
    """Brute force without a budget (K unbounded): recursion over each non-empty cell from
    the root cells, the same statistics computed directly from the cell's points. Returns
    the leaves as (level, i, j, k) in the oracle's numbering order."""
    idx, ok = finest_cells(points, lo, root_side, roots, levels)
    q = _quantise(colors)
    thr = float(np.float32(tau)) * QMAX * QMAX
    out = {l: [] for l in range(levels)}

    def visit(l, i, j, k):
        f = 1 << (levels - 1 - l)
        inside = ok & (idx[0] // f == i) & (idx[1] // f == j) & (idx[2] // f == k)
        n = int(inside.sum())
        if n == 0:
            return
        s1 = [int(q[ch][inside].sum()) for ch in range(3)]
        s2 = [int((q[ch][inside] * q[ch][inside]).sum()) for ch in range(3)]
        v = sum(float(s2[ch]) / n - (float(s1[ch]) / n) ** 2 for ch in range(3)) / 3.0
        if l + 1 < levels and v > thr:
            for dk in (0, 1):
                for dj in (0, 1):
                    for di in (0, 1):
                        visit(l + 1, 2 * i + di, 2 * j + dj, 2 * k + dk)
        else:
            out[l].append((l, i, j, k))

    for k in range(roots[2]):
        for j in range(roots[1]):
            for i in range(roots[0]):
                visit(0, i, j, k)
    leaves = []
    for l in range(levels):
        leaves.extend(sorted(out[l], key=lambda c: (c[3], c[2], c[1])))
    return leaves


def merge64(mu, sigma, amp, width, height, cell, sigma_max):
    """Merge of 2D particles (see the module docstring). mu [2, K], sigma [K], amp [3, K]
    (FP32). Returns (mu, sigma, amp) of the output particles (FP32) and the group of every
    input particle (-1 if it does not take part)."""
    mu = np.asarray(mu, dtype=np.float32)
    sigma = np.asarray(sigma, dtype=np.float32)
    amp = np.asarray(amp, dtype=np.float32)
    K = sigma.shape[0]
    cell = float(np.float32(cell))
    gx = int(np.ceil(width / cell))
    with np.errstate(invalid="ignore"):
        ok = (np.isfinite(mu).all(axis=0) & np.isfinite(sigma) & np.isfinite(amp).all(axis=0) & (sigma > 0)
              & (sigma <= np.float32(sigma_max)))
        m64 = mu.astype(np.float64)
        ok &= (m64[0] >= 0) & (m64[0] < width) & (m64[1] >= 0) & (m64[1] < height)
        cx = np.floor(m64[0] / cell)
        cy = np.floor(m64[1] / cell)
    key = np.where(ok, cy * gx + cx, -1).astype(np.int64)
    members = {}
    for k in range(K):
        if key[k] >= 0:
            members.setdefault(int(key[k]), []).append(k)
    leader = {}
    for c, ks in members.items():
        if len(ks) >= 2:
            for k in ks:
                leader[k] = ks[0]
    out_mu, out_s, out_a = [], [], []
    for k in range(K):
        if k in leader and leader[k] != k:
            continue
        if k in leader:
            ks = members[int(key[k])]
            w = sigma[ks].astype(np.float64) ** 2
            W = float(w.sum())
            out_mu.append((mu[:, ks].astype(np.float64) * w[None, :]).sum(axis=1) / W)
            out_s.append(np.sqrt(W))
            out_a.append((amp[:, ks].astype(np.float64) * w[None, :]).sum(axis=1) / W)
        else:
            out_mu.append(mu[:, k].astype(np.float64))
            out_s.append(float(sigma[k]))
            out_a.append(amp[:, k].astype(np.float64))
    if not out_s:
        return np.zeros((2, 0), np.float32), np.zeros(0, np.float32), np.zeros((3, 0), np.float32), key
    return (np.stack(out_mu, axis=1).astype(np.float32), np.asarray(out_s).astype(np.float32),
            np.stack(out_a, axis=1).astype(np.float32), key)
