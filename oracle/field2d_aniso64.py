"""FP64 oracle of the 2D kernel-sum representation with anisotropic kernels: the variant the
paper's Table 2 times against its isotropic one (settings (D, K) of the 2D fit).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never calls
it and shares no code, constants table or helper with it.

    f_c(x) = sum over k with |x - mu_k| < D of A_kc exp(-(x - mu_k)^T Sigma_k^-1 (x - mu_k))

with the 2D form of eq. 6, Sigma_k = R(theta_k) diag(s1_k^2, s2_k^2) R(theta_k)^T,
R(theta) = [[cos, -sin], [sin, cos]], and the kernel of eq. 5 (no factor 1/2, as eq. 8):
its inverse (the conic) is
    P00 = c^2 / s1^2 + s^2 / s2^2,  P01 = c s (1/s1^2 - 1/s2^2),  P11 = s^2 / s1^2 + c^2 / s2^2
(c = cos theta, s = sin theta), and the exponent is P00 dx^2 + 2 P01 dx dy + P11 dy^2. The
support, pixel grid, invalid particles (non-finite parameters, a scale <= 0, or a conic
entry overflowing in FP32) and the order of the sum are those of the isotropic field
(oracle/field2d64.py): with s1 = s2 = sigma it is that field for any theta.

Gradients of L with w_c(x) = dL/df_c(x) and t(x) = (sum_c w_c A_kc) g_k(x):
    dL/dA_kc = sum_x w_c g_k
    dL/dmu_x = sum_x 2 t (P00 dx + P01 dy),  dL/dmu_y = sum_x 2 t (P01 dx + P11 dy)
    dL/dP00 = -sum_x t dx^2, dL/dP01 = -2 sum_x t dx dy, dL/dP11 = -sum_x t dy^2
and through the conic's formula to theta, s1, s2.
"""
from __future__ import annotations

import math

import numpy as np

from . import field2d64 as F

CHANNELS = 3


def conic(theta, scale):
    """(P00, P01, P11) of R(theta) diag(s1^2, s2^2) R(theta)^T inverted, FP64 [3, K]."""
    th = np.asarray(theta, dtype=np.float64)
    s = np.asarray(scale, dtype=np.float64)
    c, sn = np.cos(th), np.sin(th)
    i1, i2 = 1.0 / (s[0] * s[0]), 1.0 / (s[1] * s[1])
    return np.array([c * c * i1 + sn * sn * i2, c * sn * (i1 - i2), sn * sn * i1 + c * c * i2])


def _valid(mu, theta, scale, amp):
    mu = np.asarray(mu, dtype=np.float32)
    theta = np.asarray(theta, dtype=np.float32)
    scale = np.asarray(scale, dtype=np.float32)
    amp = np.asarray(amp, dtype=np.float32)
    with np.errstate(all="ignore"):
        P = conic(theta, scale)
        P32 = P.astype(np.float32)
    ok = (np.isfinite(mu).all(axis=0) & np.isfinite(theta) & np.isfinite(scale).all(axis=0)
          & (scale > 0).all(axis=0) & np.isfinite(amp).all(axis=0) & np.isfinite(P32).all(axis=0))
    return mu, theta, scale, amp, P, ok


def _footprint(k, mu, P, support, width, height):
    x0, x1, y0, y1 = F._window(mu[0, k], mu[1, k], support, width, height)
    if x1 < x0 or y1 < y0:
        return None
    cols = np.arange(x0, x1 + 1)
    rows = np.arange(y0, y1 + 1)
    px = (cols.astype(np.float32) + np.float32(0.5))[None, :]
    py = (rows.astype(np.float32) + np.float32(0.5))[:, None]
    inside = F.support_mask_f32(px, py, mu[0, k], mu[1, k], support)
    if not inside.any():
        return None
    dx = px.astype(np.float64) - float(mu[0, k])
    dy = py.astype(np.float64) - float(mu[1, k])
    a, b, c = P[:, k]
    g = np.exp(-(a * dx * dx + 2.0 * b * dx * dy + c * dy * dy)) * inside
    return rows, cols, dx, dy, g


def render_field_aniso64(mu, theta, scale, amp, width, height, support):
    """The image [3][H][W] (FP64), particles added in index order."""
    mu, theta, scale, amp, P, ok = _valid(mu, theta, scale, amp)
    img = np.zeros((CHANNELS, height, width))
    for k in np.nonzero(ok)[0]:
        fp = _footprint(k, mu, P, support, width, height)
        if fp is None:
            continue
        rows, cols, _, _, g = fp
        for ch in range(CHANNELS):
            img[ch, rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1] += float(amp[ch, k]) * g
    return img


def field_aniso_grads64(mu, theta, scale, amp, width, height, support, dL_dimage):
    """(dL/dmu [2][K], dL/dtheta [K], dL/dscale [2][K], dL/dA [3][K]) in FP64."""
    mu, theta, scale, amp, P, ok = _valid(mu, theta, scale, amp)
    w = np.asarray(dL_dimage, dtype=np.float64)
    K = theta.shape[0]
    gmu, gth, gsc, gamp = np.zeros((2, K)), np.zeros(K), np.zeros((2, K)), np.zeros((CHANNELS, K))
    for k in np.nonzero(ok)[0]:
        fp = _footprint(k, mu, P, support, width, height)
        if fp is None:
            continue
        rows, cols, dx, dy, g = fp
        wk = w[:, rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1]
        for ch in range(CHANNELS):
            gamp[ch, k] = float((wk[ch] * g).sum())
        t = sum(wk[ch] * float(amp[ch, k]) for ch in range(CHANNELS)) * g
        a, b, c = P[:, k]
        gmu[0, k] = float((2.0 * t * (a * dx + b * dy)).sum())
        gmu[1, k] = float((2.0 * t * (b * dx + c * dy)).sum())
        ga, gb, gc = -float((t * dx * dx).sum()), -2.0 * float((t * dx * dy).sum()), -float((t * dy * dy).sum())
        th, s1, s2 = float(theta[k]), float(scale[0, k]), float(scale[1, k])
        cs, sn = math.cos(th), math.sin(th)
        i1, i2 = 1.0 / (s1 * s1), 1.0 / (s2 * s2)
        # P00 = c^2 i1 + s^2 i2, P01 = c s (i1 - i2), P11 = s^2 i1 + c^2 i2
        dth = (ga * 2.0 * cs * sn * (i2 - i1) + gb * (cs * cs - sn * sn) * (i1 - i2)
               + gc * 2.0 * cs * sn * (i1 - i2))
        d1 = -2.0 / (s1 * s1 * s1) * (ga * cs * cs + gb * cs * sn + gc * sn * sn)
        d2 = -2.0 / (s2 * s2 * s2) * (ga * sn * sn - gb * cs * sn + gc * cs * cs)
        gth[k], gsc[0, k], gsc[1, k] = dth, d1, d2
    return gmu, gth, gsc, gamp


def field_aniso_footprints_f32(mu, theta, scale, amp, width, height, support):
    """Binning view: every valid particle a disk of radius D around mu, depth 1."""
    mu, theta, scale, amp, P, ok = _valid(mu, theta, scale, amp)
    K = theta.shape[0]
    r = np.where(ok, np.float32(support), np.float32(0.0)).astype(np.float32)
    return {"u": mu[0].copy(), "v": mu[1].copy(), "z": np.ones(K, np.float32), "r": r,
            "width": width, "height": height}
