"""FP64 oracle of the quadtree initialisation and the multiscale edits of 2D particles
(the paper's Section 3, "Initial with Tree Structure", and Section 2, "Multiscale").

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never calls
it and shares no code, constants table or helper with it.

Quadtree initialisation. The paper places particles at the leaves of a quadtree over
the image: a leaf cell carries the average colour of its pixels and a scale of half the
cell width. It does not say when a cell splits or how the particle count is bounded;
the readings here:

* the image is covered by a grid of square root cells of side `root` pixels (a power of
  two; cells at the right and bottom borders are clipped to the image; the budget K
  allows at least one particle per root cell); a cell of side `side` splits
  into its four quadrants (side / 2, quadrants outside the image dropped) when its colour
  variance exceeds `tau` and side / 2 >= `min_side`. The colour variance is the mean over
  the channels of the population variance of the cell's in-image pixels;
* the tree grows level by level; the particle budget K is kept by refusing a whole
  level: if splitting every splittable cell of a level would bring the number of cells
  that can still become leaves above K (leaves so far + cells of the level that do not
  split + 4 x the splitting ones, counting only in-image quadrants), no cell of that
  level splits and every cell of it becomes a leaf;
* leaves are numbered level by level (root level first), row-major within a level; a
  leaf's particle: centre = the centre of its in-image rectangle, sigma = side / 2,
  amplitude = the mean colour of its pixels (FP64, rounded to FP32).

Multiscale edits (Section 2: isotropic kernels are easily divided or deleted according
to their scale; the readings):

* prune: drop particles whose largest amplitude magnitude max_c |A_kc| is below
  `amp_min` (FP32 comparison), and particles with a non-finite parameter or sigma <= 0;
  the others keep their order;
* split: a particle with sigma > `sigma_max` is replaced, in place, by four particles of
  scale sigma / 2 centred at mu + (-sigma/2, -sigma/2), (+sigma/2, -sigma/2),
  (-sigma/2, +sigma/2), (+sigma/2, +sigma/2) (FP32 sums, one rounding each), with the same
  amplitude; the others are copied.

Pins (tests/test_tree2d_oracle.py): a flat image gives one particle per root cell with
its colour; a single bright pixel refines only the cells on its path; the budget rule;
the amplitude sum rule (the leaves' pixel-weighted mean colour is the image mean);
prune and split on hand-made particle sets.
"""
from __future__ import annotations

import numpy as np


def _cell_rect(x0, y0, side, width, height):
    return x0, y0, min(x0 + side, width), min(y0 + side, height)


def quadtree_init64(target, K, root=64, min_side=2, tau=1e-3, return_stats=False):
    """Particles (mu [2][n], sigma [n], amp [3][n]) of the quadtree leaves of `target`
    [3][H][W]; with `return_stats`, also the colour variance of every visited cell, per
    level (for the tests' margin checks)."""
    assert root >= 1 and root & (root - 1) == 0 and min_side >= 1, "root must be a power of two"
    img = np.asarray(target, dtype=np.float64)
    C, H, W = img.shape
    cells = [(x, y) for y in range(0, H, root) for x in range(0, W, root)]
    assert K >= len(cells), "the budget must allow one particle per root cell"
    side = root
    leaves = []          # (x0, y0, side, mean colour)
    seen = []
    while cells:
        stats = []
        for (x, y) in cells:
            x0, y0, x1, y1 = _cell_rect(x, y, side, W, H)
            block = img[:, y0:y1, x0:x1].reshape(C, -1)
            stats.append((block.mean(axis=1), float(block.var(axis=1).mean())))
        seen.append([v for _, v in stats])
        half = side // 2
        can = [v > tau and half >= min_side for _, v in stats]
        kids = []
        for (x, y), c in zip(cells, can):
            if c:
                kids.append([(x + dx, y + dy) for dy in (0, half) for dx in (0, half) if x + dx < W and y + dy < H])
            else:
                kids.append(None)
        potential = len(leaves) + sum(1 for k in kids if k is None) + sum(len(k) for k in kids if k is not None)
        if potential > K:
            kids = [None] * len(cells)
        nxt = []
        for (x, y), (mean, _), k in zip(cells, stats, kids):
            if k is None:
                leaves.append((x, y, side, mean))
            else:
                nxt.extend(k)
        # the next level, row-major
        cells = sorted(nxt, key=lambda c: (c[1], c[0]))
        side = half
    n = len(leaves)
    mu = np.zeros((2, n))
    sigma = np.zeros(n)
    amp = np.zeros((C, n))
    for i, (x, y, s, mean) in enumerate(leaves):
        x0, y0, x1, y1 = _cell_rect(x, y, s, W, H)
        mu[:, i] = (0.5 * (x0 + x1), 0.5 * (y0 + y1))
        sigma[i] = 0.5 * s
        amp[:, i] = mean
    out = (mu.astype(np.float32), sigma.astype(np.float32), amp.astype(np.float32))
    return (out, seen) if return_stats else out


def prune64(mu, sigma, amp, amp_min):
    mu = np.asarray(mu, np.float32)
    sigma = np.asarray(sigma, np.float32)
    amp = np.asarray(amp, np.float32)
    ok = np.isfinite(mu).all(axis=0) & np.isfinite(sigma) & (sigma > 0) & np.isfinite(amp).all(axis=0)
    with np.errstate(invalid="ignore"):
        keep = ok & (np.abs(amp).max(axis=0) >= np.float32(amp_min))
    return mu[:, keep], sigma[keep], amp[:, keep]


def split64(mu, sigma, amp, sigma_max):
    mu = np.asarray(mu, np.float32)
    sigma = np.asarray(sigma, np.float32)
    amp = np.asarray(amp, np.float32)
    out_mu, out_s, out_a = [], [], []
    for k in range(sigma.shape[0]):
        if sigma[k] > np.float32(sigma_max):
            h = sigma[k] / np.float32(2.0)
            for sy in (-1, 1):
                for sx in (-1, 1):
                    out_mu.append((mu[0, k] + np.float32(sx) * h, mu[1, k] + np.float32(sy) * h))
                    out_s.append(h)
                    out_a.append(amp[:, k])
        else:
            out_mu.append((mu[0, k], mu[1, k]))
            out_s.append(sigma[k])
            out_a.append(amp[:, k])
    if not out_s:
        return np.zeros((2, 0), np.float32), np.zeros(0, np.float32), np.zeros((3, 0), np.float32)
    return (np.asarray(out_mu, np.float32).T.copy(), np.asarray(out_s, np.float32),
            np.asarray(out_a, np.float32).T.copy())
