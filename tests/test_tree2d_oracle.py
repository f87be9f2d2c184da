"""Pins of the FP64 oracle of the quadtree initialisation and the multiscale edits.

Each test names the oracle mistake it is there to catch; none compares the oracle with
itself.
"""
import numpy as np
import pytest

from oracle import tree2d64 as T


def test_flat_image_gives_one_particle_per_root_cell():
    # catches: splitting a uniform cell, wrong centres of clipped border cells, sigma not
    # half the cell width, leaves out of row-major order
    img = np.empty((3, 70, 100), np.float32)
    img[:] = np.float32([0.2, 0.4, 0.6])[:, None, None]
    mu, s, a = T.quadtree_init64(img, K=1000, root=32, min_side=2, tau=1e-6)
    assert s.shape == (12,) and np.all(s == 16.0)
    np.testing.assert_allclose(a, np.repeat(np.float32([[0.2], [0.4], [0.6]]), 12, axis=1), rtol=1e-7)
    xs = [16.0, 48.0, 80.0, 98.0]
    ys = [16.0, 48.0, 67.0]
    np.testing.assert_array_equal(mu[0], np.tile(xs, 3))
    np.testing.assert_array_equal(mu[1], np.repeat(ys, 4))


def test_single_bright_pixel_refines_only_its_path():
    # catches: splitting cells with zero variance, a wrong quadrant order, min_side off by
    # one level
    img = np.zeros((3, 64, 64), np.float32)
    img[:, 21, 37] = 1.0
    mu, s, a = T.quadtree_init64(img, K=1000, root=64, min_side=2, tau=1e-9)
    # three quiet siblings at each of the sides 32, 16, 8, 4, then the four cells of side 2
    assert s.shape == (16,)
    assert sorted(s.tolist()) == [1.0] * 4 + [2.0] * 3 + [4.0] * 3 + [8.0] * 3 + [16.0] * 3
    k = int(np.nonzero((s == 1.0) & (a[0] > 0))[0][0])
    assert a[0, k] == pytest.approx(0.25) and tuple(mu[:, k]) == (37.0, 21.0)
    # the side-2 cells are the four quadrants of the 4-pixel cell at (36, 20), row-major
    fine = np.nonzero(s == 1.0)[0]
    assert [tuple(mu[:, i]) for i in fine] == [(37.0, 21.0), (39.0, 21.0), (37.0, 23.0), (39.0, 23.0)]


def test_budget_refuses_a_whole_level():
    # catches: a budget that cuts a level part way, or that is checked after splitting
    img = np.zeros((3, 64, 64), np.float32)
    img[:, 21, 37] = 1.0
    mu, s, a = T.quadtree_init64(img, K=10, root=64, min_side=2, tau=1e-9)
    assert s.shape == (10,)
    assert sorted(s.tolist()) == [4.0] * 4 + [8.0] * 3 + [16.0] * 3


def test_leaf_colours_average_to_the_image_mean():
    # catches: a mean over the nominal rather than the in-image area of border cells, a
    # leaf lost or counted twice
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 1, (3, 75, 90)).astype(np.float32)
    mu, s, a = T.quadtree_init64(img, K=5000, root=32, min_side=2, tau=0.05)
    # the pixel count of each leaf from its centre and its (clipped) side
    side = 2 * s.astype(np.float64)
    x0 = np.floor(mu[0] - side / 2 + 1e-9)
    x0 = np.where(mu[0] + side / 2 > 90, mu[0] - (90 - mu[0]), x0)
    w = np.minimum(side, 2 * (mu[0] - x0))
    y0 = np.floor(mu[1] - side / 2 + 1e-9)
    y0 = np.where(mu[1] + side / 2 > 75, mu[1] - (75 - mu[1]), y0)
    h = np.minimum(side, 2 * (mu[1] - y0))
    area = w * h
    assert area.sum() == 75 * 90
    np.testing.assert_allclose((a.astype(np.float64) * area).sum(axis=1), img.astype(np.float64).sum(axis=(1, 2)),
                               rtol=1e-6)


def test_prune_and_split():
    # catches: pruning on a signed amplitude, losing order, children placed at +-sigma
    # instead of +-sigma/2, scales not halved
    mu = np.float32([[1, 2, 3, 4, 5], [10, 20, 30, 40, 50]])
    s = np.float32([1.0, 2.0, -1.0, 3.0, 0.5])
    a = np.float32([[0.5, 0.01, 0.9, -0.3, 0.02], [0, 0, 0, 0, -0.06], [0, 0.02, 0, 0, 0]])
    pm, ps, pa = T.prune64(mu, s, a, 0.05)
    np.testing.assert_array_equal(ps, np.float32([1.0, 3.0, 0.5]))
    np.testing.assert_array_equal(pm[0], np.float32([1, 4, 5]))
    sm, ss, sa = T.split64(np.float32([[10, 7], [20, 8]]), np.float32([4.0, 1.0]), np.float32([[1, 2], [3, 4], [5, 6]]),
                           2.0)
    np.testing.assert_array_equal(sm, np.float32([[8, 12, 8, 12, 7], [18, 18, 22, 22, 8]]))
    np.testing.assert_array_equal(ss, np.float32([2, 2, 2, 2, 1]))
    np.testing.assert_array_equal(sa, np.float32([[1, 1, 1, 1, 2], [3, 3, 3, 3, 4], [5, 5, 5, 5, 6]]))
