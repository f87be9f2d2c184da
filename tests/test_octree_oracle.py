"""Pins of the octree initialisation (3D) and of the merge of 2D particles (oracle/octree64.py)
against closed forms, a brute-force recursion and exact invariants."""
import numpy as np
import pytest

from oracle import octree64 as OT
from oracle import tree2d64 as T2
import scenegen as S

LO = (-1.0, -1.0, -1.0)


def test_uniform_cloud_in_one_root_cell_is_one_particle():
    rng = np.random.default_rng(0)
    pts = rng.uniform(-0.99, -0.01, (3, 500)).astype(np.float32)      # inside root cell (0, 0, 0)
    col = np.tile(np.array([[0.25], [0.5], [0.75]], np.float32), (1, 500))
    out = OT.octree_init64(pts, col, LO, 1.0, (2, 2, 2), 4, 1e-4, 100, opacity=0.3)
    assert out["count"] == 1
    np.testing.assert_array_equal(out["pos"][:, 0], np.float32([-0.5, -0.5, -0.5]))
    assert out["scale"][0] == np.float32(0.5) and out["opacity"][0] == np.float32(0.3)
    np.testing.assert_array_equal(out["color"][:, 0], (np.rint(np.float64([0.25, 0.5, 0.75]) * 65535) / 65535)
                                  .astype(np.float32))


def test_two_colours_split_once_into_their_octants():
    """Red points in octant (0,0,0) and blue in octant (1,1,1) of one root cell: the cell
    splits once; the six empty octants carry no particle; each half's colour is exact."""
    rng = np.random.default_rng(1)
    a = rng.uniform(-0.99, -0.51, (3, 200))
    b = rng.uniform(-0.49, -0.01, (3, 300))
    pts = np.concatenate([a, b], axis=1).astype(np.float32)
    col = np.concatenate([np.tile([[1.0], [0.0], [0.0]], (1, 200)), np.tile([[0.0], [0.0], [1.0]], (1, 300))],
                         axis=1).astype(np.float32)
    out = OT.octree_init64(pts, col, LO, 1.0, (2, 2, 2), 3, 1e-3, 100)
    assert out["count"] == 2
    np.testing.assert_array_equal(out["pos"].T, np.float32([[-0.75, -0.75, -0.75], [-0.25, -0.25, -0.25]]))
    np.testing.assert_array_equal(out["scale"], np.float32([0.25, 0.25]))
    np.testing.assert_array_equal(out["color"].T, np.float32([[1, 0, 0], [0, 0, 1]]))


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_levelwise_tree_equals_recursive_brute_force(seed):
    """Without a binding budget the level-by-level tree is the plain recursion: split a
    non-empty cell while its variance exceeds tau (statistics from its own points)."""
    pts, col = S.point_cloud(3000, seed=seed, extent=0.95)
    levels, roots, tau = 4, (2, 2, 2), 2e-3
    out = OT.octree_init64(pts, col, LO, 1.0, roots, levels, tau, 10 ** 9)
    ref = OT.octree_init_recursive(pts, col, LO, 1.0, roots, levels, tau)
    assert out["count"] == len(ref) > 8
    edge = np.float64(1.0) / (1 << np.array([c[0] for c in ref]))
    centre = np.array([[c[1], c[2], c[3]] for c in ref], np.float64).T
    np.testing.assert_array_equal(out["pos"], (np.float64(-1.0) + (centre + 0.5) * edge).astype(np.float32))
    np.testing.assert_array_equal(out["scale"], (0.5 * edge).astype(np.float32))


def test_leaves_partition_the_points_and_keep_the_colour_sums():
    """Every in-grid point lies in exactly one leaf; the leaves' point-weighted colour sums
    (exact integers) add up to the cloud's."""
    pts, col = S.point_cloud(4000, seed=5, extent=1.2)       # some points outside the grid
    levels, roots = 4, (2, 2, 2)
    out = OT.octree_init64(pts, col, LO, 1.0, roots, levels, 1e-3, 10 ** 9)
    stats = OT.level_stats(pts, col, LO, 1.0, roots, levels)
    idx, ok = OT.finest_cells(pts, LO, 1.0, roots, levels)
    assert 0 < ok.sum() < pts.shape[1]
    owner = np.full(pts.shape[1], -1)
    for p, (c, h) in enumerate(zip(out["pos"].T.astype(np.float64), out["scale"].astype(np.float64))):
        inside = ok & np.all(np.abs(pts.astype(np.float64) - c[:, None]) <= h + 1e-12, axis=0)
        # a point on a shared face belongs to the cell its finest index falls in
        f = 2 * h / (1.0 / (1 << (levels - 1)))
        cell = np.floor((c[:, None] - h - np.float64(-1.0)) / (2 * h)).astype(np.int64)
        inside &= np.all(idx // int(round(f)) == cell, axis=0)
        assert (owner[inside] == -1).all()
        owner[inside] = p
    assert (owner[ok] >= 0).all() and (owner[~ok] == -1).all()
    q = np.rint(np.clip(col.astype(np.float64), 0, 1) * 65535).astype(np.int64)
    n0, S1, _ = stats[0]
    for ch in range(3):
        assert S1[ch].sum() == q[ch][ok].sum()


def test_budget_refuses_a_whole_level():
    pts, col = S.point_cloud(3000, seed=6, extent=0.95)
    levels, roots, tau = 4, (2, 2, 2), 1e-4
    free = OT.octree_init64(pts, col, LO, 1.0, roots, levels, tau, 10 ** 9)
    ref = OT.octree_init_recursive(pts, col, LO, 1.0, roots, levels, tau)
    per_level = np.bincount([c[0] for c in ref], minlength=levels)
    assert per_level[-1] > 0
    # a budget just below the full tree refuses some level: fewer particles, none finer than it
    cut = OT.octree_init64(pts, col, LO, 1.0, roots, levels, tau, free["count"] - 1)
    assert cut["count"] <= free["count"] - 1
    assert cut["scale"].min() > free["scale"].min()
    # a budget of the root cells only: the root level itself refuses
    root = OT.octree_init64(pts, col, LO, 1.0, roots, levels, tau, 8)
    assert root["count"] == 8 and (root["scale"] == np.float32(0.5)).all()


def _parents(n, cell, seed):
    rng = np.random.default_rng(seed)
    gx = 512 // cell
    cells = rng.choice(gx * gx, size=n, replace=False)
    mu = np.stack([(cells % gx + 0.5) * cell, (cells // gx + 0.5) * cell]).astype(np.float32)
    sigma = np.full(n, np.float32(cell / 2))
    amp = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    return mu, sigma, amp


def test_merge_undoes_split():
    mu, sigma, amp = _parents(60, 8, 7)
    cmu, cs, ca = T2.split64(mu, sigma, amp, 1.0)
    assert cs.shape[0] == 240
    mmu, ms, ma, key = OT.merge64(cmu, cs, ca, 512, 512, 8, 2.0)
    assert ms.shape[0] == 60
    np.testing.assert_array_equal(mmu, mu)
    np.testing.assert_array_equal(ms, sigma)
    np.testing.assert_allclose(ma, amp, rtol=2 ** -23, atol=2 ** -24)


def test_merge_keeps_singletons_order_and_mass():
    rng = np.random.default_rng(8)
    K = 400
    mu = rng.uniform(0, 128, (2, K)).astype(np.float32)
    sigma = rng.uniform(0.2, 3.0, K).astype(np.float32)
    amp = rng.normal(0, 1, (3, K)).astype(np.float32)
    sigma[5] = np.nan
    mu[0, 9] = -3.0
    mmu, ms, ma, key = OT.merge64(mu, sigma, amp, 128, 128, 16, 1.5)
    part = key >= 0
    assert not part[5] and not part[9] and not part[sigma > 1.5].any()
    groups = {}
    for k in np.nonzero(part)[0]:
        groups.setdefault(int(key[k]), []).append(k)
    merged = {g[0]: g for g in groups.values() if len(g) >= 2}
    gone = {k for g in merged.values() for k in g[1:]}
    survivors = [k for k in range(K) if k not in gone]
    assert ms.shape[0] == len(survivors) < K
    for o, k in enumerate(survivors):
        if k not in merged:
            assert (mmu[:, o] == mu[:, k]).all() and (ms[o] == sigma[k] or np.isnan(sigma[k]))
            assert (ma[:, o] == amp[:, k]).all()
        else:
            g = merged[k]
            w = sigma[g].astype(np.float64) ** 2
            assert abs(float(ms[o]) ** 2 - w.sum()) <= 1e-6 * w.sum()
            # per channel the kernel mass pi A sigma^2 is kept
            np.testing.assert_allclose(ma[:, o].astype(np.float64) * float(ms[o]) ** 2,
                                       (amp[:, g].astype(np.float64) * w).sum(axis=1), rtol=1e-6, atol=1e-6)
            lo = np.floor(mu[:, g].astype(np.float64) / 16).min(axis=1) * 16
            assert np.all(mmu[:, o] >= lo) and np.all(mmu[:, o] <= lo + 16)
