"""Pins of the FP64 SSIM oracle (the SSIM term of the paper's loss).

Each test names the oracle mistake it is there to catch; none compares the oracle with
itself.
"""
import math

import numpy as np
import pytest

from oracle import ssim64 as Q


def test_window():
    # catches: a window of the wrong width or sigma, or one that is not normalised
    g = Q.gaussian_window()
    assert g.shape == (11,) and g.sum() == pytest.approx(1.0, abs=1e-15)
    assert g[5] / g[6] == pytest.approx(math.exp(1.0 / (2 * 1.5 ** 2)), rel=1e-14)
    assert g[0] / g[5] == pytest.approx(math.exp(-25.0 / 4.5), rel=1e-14)


def test_identical_images_and_symmetry():
    # catches: a wrong stabiliser, a missing factor 2, a numerator/denominator swap
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (3, 20, 17))
    y = rng.uniform(0, 1, (3, 20, 17))
    assert Q.ssim64(x, x) == pytest.approx(1.0, abs=1e-14)
    assert Q.ssim64(x, y) == pytest.approx(Q.ssim64(y, x), abs=1e-14)
    assert Q.ssim64(x, y) < 0.9
    np.testing.assert_allclose(Q.ssim_grad64(x, x), 0.0, atol=1e-15)   # a maximum


def test_constant_images_closed_form():
    # catches: variance terms computed without subtracting the mean, C1 and C2 swapped;
    # away from the borders two constant images have mu = c, s^2 = s_xy = 0
    c1, c2 = 0.3, 0.7
    x = np.full((1, 30, 30), c1)
    y = np.full((1, 30, 30), c2)
    S = Q.ssim_map64(x, y)
    want = (2 * c1 * c2 + Q.C1) / (c1 * c1 + c2 * c2 + Q.C1)
    np.testing.assert_allclose(S[0, 5:25, 5:25], want, rtol=1e-12)
    # at a corner the zero padding shows: the window sees only a quarter of the image
    assert abs(S[0, 0, 0] - want) > 1e-3


def test_brute_force_window_on_a_tiny_image():
    # catches: a filter applied along one axis only, a shifted window, edge padding
    # instead of zeros
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (1, 9, 13))
    y = rng.uniform(0, 1, (1, 9, 13))
    g = Q.gaussian_window()
    H, W = 9, 13
    S = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            st = np.zeros(5)
            for a in range(-5, 6):
                for b in range(-5, 6):
                    ii, jj = i + a, j + b
                    if 0 <= ii < H and 0 <= jj < W:
                        wgt = g[a + 5] * g[b + 5]
                        xv, yv = x[0, ii, jj], y[0, ii, jj]
                        st += wgt * np.array([xv, yv, xv * xv, yv * yv, xv * yv])
            mx, my, exx, eyy, exy = st
            vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
            S[i, j] = ((2 * mx * my + Q.C1) * (2 * cxy + Q.C2)) / ((mx * mx + my * my + Q.C1) * (vx + vy + Q.C2))
    np.testing.assert_allclose(Q.ssim_map64(x, y)[0], S, rtol=1e-12, atol=1e-14)


def test_gradient_matches_central_differences():
    # catches: a dropped chain-rule term (through s_x^2 or s_xy), the filter not
    # transposed back, the mean's 1/N missing, the loss's sign
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (2, 12, 14))
    y = rng.uniform(0, 1, (2, 12, 14))
    g = Q.ssim_grad64(x, y)
    _, gl = Q.l1_ssim_loss64(x, y)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 5, 7), (0, 11, 13), (1, 3, 0), (0, 6, 6)]:
        p, m = x.copy(), x.copy()
        p[idx] += h
        m[idx] -= h
        fd = (Q.ssim64(p, y) - Q.ssim64(m, y)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-11)
        fdl = (Q.l1_ssim_loss64(p, y)[0] - Q.l1_ssim_loss64(m, y)[0]) / (2 * h)
        assert gl[idx] == pytest.approx(fdl, rel=1e-6, abs=1e-11)
