"""Pins of the FP64 oracle of the 2D kernel-sum representation (Section 3, eq. 2, eq. 8).

Each test names the oracle mistake it is there to catch; none compares the oracle with
itself.
"""
import math

import numpy as np
import pytest

from oracle import field2d64 as F
import oracle as O


def one(mu, sigma, amp):
    return (np.asarray(mu, np.float32).reshape(2, 1), np.asarray([sigma], np.float32),
            np.asarray(amp, np.float32).reshape(3, 1))


def test_single_particle_on_the_grid():
    # catches: a factor 1/2 or a normalisation in the kernel, a non-strict support test,
    # pixel centres at integers instead of half-integers, swapped x / y
    mu, s, a = one([10.5, 12.5], 2.0, [1.0, 0.5, -2.0])
    img = F.render_field64(mu, s, a, 24, 20, support=3.0)
    A = np.array([1.0, 0.5, -2.0])
    np.testing.assert_allclose(img[:, 12, 10], A, rtol=0, atol=1e-15)              # at the centre
    np.testing.assert_allclose(img[:, 12, 12], A * math.exp(-1.0), rtol=1e-15)      # one sigma along x
    np.testing.assert_allclose(img[:, 13, 11], A * math.exp(-0.5), rtol=1e-15)      # d^2 = 2
    np.testing.assert_allclose(img[:, 14, 10], A * math.exp(-1.0), rtol=1e-15)      # one sigma along y
    assert np.all(img[:, 12, 13] == 0.0) and np.all(img[:, 15, 10] == 0.0)          # d = D exactly: outside
    np.testing.assert_allclose(img[:, 14, 12], A * math.exp(-2.0), rtol=1e-15)      # d^2 = 8 < 9: inside
    # nothing outside the disk of radius 3 around the centre
    yy, xx = np.mgrid[0:20, 0:24]
    d2 = (xx + 0.5 - 10.5) ** 2 + (yy + 0.5 - 12.5) ** 2
    assert np.all(img[:, d2 >= 9.0] == 0.0)
    assert np.all(img[0, d2 < 9.0] > 0.0)


def test_lattice_sum_is_pi_sigma_squared():
    # catches: exp(-d^2 / (2 sigma^2)) (sum 2 pi sigma^2) or a kernel normalised to 1;
    # the sum of exp(-|x - mu|^2 / sigma^2) over a unit lattice equals pi sigma^2 up to
    # terms of order exp(-pi^2 sigma^2) (Poisson summation)
    for sigma, mu in ((4.0, (64.3, 63.7)), (2.5, (40.0, 41.25))):
        m, s, a = one(mu, sigma, [1.0, 2.0, 0.0])
        img = F.render_field64(m, s, a, 128, 128, support=60.0)
        assert img[0].sum() == pytest.approx(math.pi * sigma * sigma, rel=1e-12)
        assert img[1].sum() == pytest.approx(2.0 * math.pi * sigma * sigma, rel=1e-12)


def test_superposition_and_translation():
    # catches: state carried between particles, a window clipped at the wrong edge
    rng = np.random.default_rng(3)
    K, W, H, D = 40, 96, 80, 7.0
    # centres on a 1/64 grid, so that the shifted centres are exact in FP32
    mu = (np.round(np.stack([rng.uniform(20, W - 20, K), rng.uniform(20, H - 20, K)]) * 64) / 64).astype(np.float32)
    s = rng.uniform(0.7, 3.0, K).astype(np.float32)
    a = rng.uniform(-1, 1, (3, K)).astype(np.float32)
    full = F.render_field64(mu, s, a, W, H, D)
    part = F.render_field64(mu[:, :15], s[:15], a[:, :15], W, H, D) + \
        F.render_field64(mu[:, 15:], s[15:], a[:, 15:], W, H, D)
    np.testing.assert_allclose(full, part, rtol=0, atol=1e-13)
    shifted = F.render_field64(mu + np.float32([[8.0], [4.0]]), s, a, W + 8, H + 4, D)
    np.testing.assert_allclose(shifted[:, 4:, 8:], full, rtol=0, atol=1e-13)


def test_matches_brute_force_over_every_pixel_and_particle():
    # catches: a support window that misses pixels, a particle dropped at the border,
    # invalid particles that still contribute
    rng = np.random.default_rng(11)
    K, W, H, D = 25, 21, 17, 4.5
    mu = np.stack([rng.uniform(-5, W + 5, K), rng.uniform(-5, H + 5, K)]).astype(np.float32)
    s = rng.uniform(0.5, 3.0, K).astype(np.float32)
    s[3] = -1.0
    s[7] = 0.0
    mu[0, 9] = np.nan
    a = rng.uniform(0, 1, (3, K)).astype(np.float32)
    img = F.render_field64(mu, s, a, W, H, D)
    ref = np.zeros((3, H, W))
    for j in range(H):
        for i in range(W):
            for k in range(K):
                if not (s[k] > 0 and np.isfinite(mu[:, k]).all()):
                    continue
                x, y = np.float32(i + 0.5), np.float32(j + 0.5)
                dx, dy = x - mu[0, k], y - mu[1, k]
                if not (dx * dx + dy * dy < np.float32(D) * np.float32(D)):
                    continue
                d2 = (float(x) - float(mu[0, k])) ** 2 + (float(y) - float(mu[1, k])) ** 2
                ref[:, j, i] += a[:, k].astype(np.float64) * math.exp(-d2 / float(s[k]) ** 2)
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-13)


def test_gradients_match_central_differences():
    # catches: a dropped factor 2, a wrong sign of (x - mu), sigma^2 instead of sigma^3,
    # channels mixed in the position gradient
    rng = np.random.default_rng(5)
    K, W, H, D = 12, 48, 40, 12.0     # D >= 5 sigma: the support edge moves nothing measurable
    mu = np.stack([rng.uniform(8, W - 8, K), rng.uniform(8, H - 8, K)])
    s = rng.uniform(0.8, 2.2, K)
    a = rng.uniform(-1, 1, (3, K))
    w = rng.normal(size=(3, H, W))

    def loss(mu_, s_, a_):
        # FP64 parameters, so the finite differences are not rounded to FP32
        img = np.zeros((3, H, W))
        yy, xx = np.mgrid[0:H, 0:W] + 0.5
        for k in range(K):
            d2 = (xx - mu_[0, k]) ** 2 + (yy - mu_[1, k]) ** 2
            g = np.exp(-d2 / s_[k] ** 2) * (d2 < D * D)
            img += a_[:, k][:, None, None] * g
        return float((w * img).sum())

    # the analytic gradients at FP32-representable parameters
    mu32, s32, a32 = mu.astype(np.float32), s.astype(np.float32), a.astype(np.float32)
    gmu, gs, ga = F.field_grads64(mu32, s32, a32, W, H, D, w)
    mu, s, a = mu32.astype(np.float64), s32.astype(np.float64), a32.astype(np.float64)
    h = 1e-6
    for k in range(K):
        for d in range(2):
            p, m = mu.copy(), mu.copy()
            p[d, k] += h
            m[d, k] -= h
            fd = (loss(p, s, a) - loss(m, s, a)) / (2 * h)
            assert gmu[d, k] == pytest.approx(fd, rel=1e-6, abs=1e-7)
        p, m = s.copy(), s.copy()
        p[k] += h
        m[k] -= h
        assert gs[k] == pytest.approx((loss(mu, p, a) - loss(mu, m, a)) / (2 * h), rel=1e-6, abs=1e-7)
        for c in range(3):
            p, m = a.copy(), a.copy()
            p[c, k] += h
            m[c, k] -= h
            assert ga[c, k] == pytest.approx((loss(mu, s, p) - loss(mu, s, m)) / (2 * h), rel=1e-6, abs=1e-7)


def test_l1_gradient_and_binning_view():
    # catches: a sign error in the L1 gradient, sign(0) != 0, mean over the wrong count;
    # invalid particles binned
    img = np.array([[[0.5, 0.2], [0.1, 0.0]]] * 3)
    tgt = np.array([[[0.25, 0.2], [0.3, 0.0]]] * 3)
    loss, g = F.l1_loss64(img, tgt)
    assert loss == pytest.approx((0.25 + 0.2) / 4)
    np.testing.assert_array_equal(g[0], np.array([[1.0, 0.0], [-1.0, 0.0]]) / 12)
    mu = np.float32([[5.0, 9.0, np.inf], [5.0, 30.0, 1.0]])
    vw = F.field_footprints_f32(mu, np.float32([1.0, 2.0, 1.0]), np.zeros((3, 3), np.float32), 40, 40, 6.0)
    bins = O.bin_sort_ref([vw])
    assert set(bins.pidx.tolist()) == {0, 1}
    # every pixel inside a particle's support lies in one of its tiles
    for k in (0, 1):
        tiles = {int(t) for t, p in zip(bins.keys >> np.uint64(32), bins.pidx) if p == k}
        yy, xx = np.nonzero(F.support_mask_f32(np.arange(40)[None, :] + 0.5, np.arange(40)[:, None] + 0.5,
                                               mu[0, k], mu[1, k], 6.0))
        assert {(y // 16) * 3 + x // 16 for y, x in zip(yy, xx)} <= tiles
