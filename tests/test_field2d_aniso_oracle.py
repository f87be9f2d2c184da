"""Pins of the anisotropic 2D kernel sum (oracle/field2d_aniso64.py): reduction to the
isotropic field for equal scales, the closed form of one axis-aligned kernel, a quarter
turn swapping the axes, the lattice sum pi s1 s2, a brute-force loop and central finite
differences of every gradient."""
import math

import numpy as np
import pytest

from oracle import field2d64 as F
from oracle import field2d_aniso64 as FA


def _random(K, W, H, seed, smin=0.8, smax=4.0):
    rng = np.random.default_rng(seed)
    mu = np.stack([rng.uniform(0, W, K), rng.uniform(0, H, K)]).astype(np.float32)
    theta = rng.uniform(-math.pi, math.pi, K).astype(np.float32)
    scale = rng.uniform(smin, smax, (2, K)).astype(np.float32)
    amp = rng.normal(0, 1, (3, K)).astype(np.float32)
    return mu, theta, scale, amp


def test_equal_scales_are_the_isotropic_field():
    mu, theta, scale, amp = _random(60, 48, 40, 1)
    scale[1] = scale[0]
    a = FA.render_field_aniso64(mu, theta, scale, amp, 48, 40, 9.0)
    b = F.render_field64(mu, scale[0], amp, 48, 40, 9.0)
    assert np.abs(a - b).max() < 1e-12
    w = np.random.default_rng(2).normal(size=(3, 40, 48))
    gmu, gth, gsc, gamp = FA.field_aniso_grads64(mu, theta, scale, amp, 48, 40, 9.0, w)
    imu, isig, iamp = F.field_grads64(mu, scale[0], amp, 48, 40, 9.0, w)
    assert np.abs(gmu - imu).max() < 1e-9 * max(1.0, np.abs(imu).max())
    assert np.abs(gamp - iamp).max() < 1e-12
    # a circle does not turn; its radius is shared by both axes
    assert np.abs(gth).max() < 1e-9 * max(1.0, np.abs(isig).max())
    np.testing.assert_allclose(gsc[0] + gsc[1], isig, rtol=1e-9, atol=1e-9)


def test_axis_aligned_kernel_closed_form():
    """theta = 0: A exp(-1) one s1 away along x and one s2 away along y."""
    mu = np.float32([[10.5], [8.5]])
    amp = np.float32([[2.0], [1.0], [-1.0]])
    img = FA.render_field_aniso64(mu, np.float32([0.0]), np.float32([[3.0], [1.0]]), amp, 24, 20, 12.0)
    a64 = amp[:, 0].astype(np.float64)
    np.testing.assert_allclose(img[:, 8, 10], a64, rtol=1e-15)
    np.testing.assert_allclose(img[:, 8, 13], a64 * math.exp(-1.0), rtol=1e-14)
    np.testing.assert_allclose(img[:, 9, 10], a64 * math.exp(-1.0), rtol=1e-14)
    np.testing.assert_allclose(img[:, 9, 13], a64 * math.exp(-2.0), rtol=1e-14)


def test_quarter_turn_swaps_the_axes():
    mu, theta, scale, amp = _random(30, 40, 40, 3)
    a = FA.render_field_aniso64(mu, np.zeros(30, np.float32), scale, amp, 40, 40, 10.0)
    b = FA.render_field_aniso64(mu, np.full(30, np.float32(math.pi / 2)), scale[::-1].copy(), amp, 40, 40, 10.0)
    assert np.abs(a - b).max() < 1e-6      # pi/2 in FP32 is within 1e-7 of a quarter turn


def test_lattice_sum_is_pi_s1_s2():
    for th in (0.0, 0.4, 1.1):
        mu = np.float32([[60.3], [58.9]])
        img = FA.render_field_aniso64(mu, np.float32([th]), np.float32([[4.0], [2.5]]), np.float32([[1], [0], [0]]),
                                      120, 120, 59.0)
        assert abs(img[0].sum() - math.pi * 4.0 * 2.5) < 1e-6


def test_brute_force_loop():
    mu, theta, scale, amp = _random(12, 20, 16, 4)
    theta[3] = np.nan
    scale[1, 5] = -1.0
    D = 6.5
    img = FA.render_field_aniso64(mu, theta, scale, amp, 20, 16, D)
    ref = np.zeros((3, 16, 20))
    for k in range(12):
        th, s1, s2 = float(theta[k]), float(scale[0, k]), float(scale[1, k])
        if not (np.isfinite(th) and s1 > 0 and s2 > 0):
            continue
        c, s = math.cos(th), math.sin(th)
        for y in range(16):
            for x in range(20):
                dx32 = np.float32(x + 0.5) - mu[0, k]
                dy32 = np.float32(y + 0.5) - mu[1, k]
                if not (dx32 * dx32 + dy32 * dy32 < np.float32(D) * np.float32(D)):
                    continue
                dx, dy = float(x + 0.5) - float(mu[0, k]), float(y + 0.5) - float(mu[1, k])
                # rotate into the kernel's axes: d' = R^T d
                u, v = c * dx + s * dy, -s * dx + c * dy
                ref[:, y, x] += amp[:, k].astype(np.float64) * math.exp(-(u * u / (s1 * s1) + v * v / (s2 * s2)))
    assert np.abs(img - ref).max() < 1e-12


def test_gradients_match_central_differences():
    """Analytic FP64 gradients against central differences of an FP64 loss written in the
    kernel's own axes (d rotated by -theta, exp(-(u^2/s1^2 + v^2/s2^2))), a form independent
    of the conic; the support (D = 18, over five times the largest scale) moves nothing
    measurable."""
    W, H, D = 40, 36, 18.0
    K = 6
    rng = np.random.default_rng(5)
    mu = np.stack([rng.uniform(12, W - 12, K), rng.uniform(12, H - 12, K)]).astype(np.float32)
    theta = rng.uniform(-math.pi, math.pi, K).astype(np.float32)
    scale = rng.uniform(1.2, 3.2, (2, K)).astype(np.float32)
    amp = rng.normal(0, 1, (3, K)).astype(np.float32)
    wt = rng.normal(size=(3, H, W))
    g = FA.field_aniso_grads64(mu, theta, scale, amp, W, H, D, wt)
    yy, xx = np.mgrid[0:H, 0:W] + 0.5

    def loss(m, t, sc, a):
        img = np.zeros((3, H, W))
        for k in range(K):
            dx, dy = xx - m[0, k], yy - m[1, k]
            c, s_ = math.cos(t[k]), math.sin(t[k])
            u, v = c * dx + s_ * dy, -s_ * dx + c * dy
            gk = np.exp(-(u * u / sc[0, k] ** 2 + v * v / sc[1, k] ** 2)) * (dx * dx + dy * dy < D * D)
            img += a[:, k][:, None, None] * gk
        return float((wt * img).sum())

    base = {"mu": mu.astype(np.float64), "theta": theta.astype(np.float64), "scale": scale.astype(np.float64),
            "amp": amp.astype(np.float64)}
    checked = 0
    for name, gi in zip(("mu", "theta", "scale", "amp"), g):
        for idx in np.ndindex(base[name].shape):
            h = 1e-6
            args = {k: v.copy() for k, v in base.items()}
            args[name][idx] += h
            lp = loss(args["mu"], args["theta"], args["scale"], args["amp"])
            args[name][idx] -= 2 * h
            lm = loss(args["mu"], args["theta"], args["scale"], args["amp"])
            fd = (lp - lm) / (2 * h)
            assert abs(fd - float(gi[idx])) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, float(gi[idx]))
            checked += 1
    assert checked == K * (2 + 1 + 2 + 3)
