"""FP64 oracle of the 2D kernel-sum representation of the paper's Section 3 ("Our Method").

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never calls
it and shares no code, constants table or helper with it.

What it computes: an image signal represented by K weighted isotropic Gaussian kernels,
with no compositing (the reconstruction equation of Section 3, the support region of
eq. 2 and the kernel of eq. 8):

    f_c(x) = sum over k with |x - mu_k| < D of A_kc exp(-|x - mu_k|^2 / sigma_k^2)

for pixel centres x = (i + 1/2, j + 1/2), channels c = 0, 1, 2, particle centre mu_k and
scale sigma_k > 0 in pixels, amplitude A_k (the particle's colour), support radius D in
pixels. Readings where the paper is silent:

* the kernel is the unnormalised exp(-d^2/sigma^2) of eq. 8 (no factor 1/2, no 1/(pi
  sigma^2)): the amplitude carries the scale; pinned by the lattice sum pi sigma^2;
* the support test |x - mu| < D is strict and is decided in FP32 one operation at a
  time (dx = x - mu_x, dy likewise, d2 = dx*dx + dy*dy, include iff d2 < D*D), the same
  decision the GPU takes on the same FP32 inputs; everything else is FP64;
* a particle with a non-finite parameter or sigma <= 0 contributes nothing (and gets
  zero gradients), and so does one whose 1/sigma^2 overflows in FP32 (sigma < ~1e-19);
* the loss of the paper's fit is read as its L1 term, mean |f - target| over channels
  and pixels (the SSIM term is not on this path); its gradient is
  sign(f - target) / numel with sign(0) = 0.

Gradients of a loss L with w_c(x) = dL/df_c(x), summed over the pixels in the support:

    dL/dA_kc  = sum_x w_c(x) g_k(x)
    dL/dmu_k  = sum_x (sum_c w_c(x) A_kc) g_k(x) 2 (x - mu_k) / sigma_k^2
    dL/dsigma = sum_x (sum_c w_c(x) A_kc) g_k(x) 2 |x - mu_k|^2 / sigma_k^3

(the support indicator has zero derivative almost everywhere). The paper's eq. 3 is the
same derivative written for its general kernel W.

Pins (tests/test_field2d_oracle.py): the closed form of one particle on the pixel grid
(value A at its centre, A/e one sigma away, 0 at exactly D), the lattice sum
pi sigma^2 of one kernel, superposition, integer translation, a brute-force double loop
over every pixel and particle on tiny inputs, and FP64 central differences of the
gradients.
"""
from __future__ import annotations

import math

import numpy as np

CHANNELS = 3


def _valid(mu, sigma, amp):
    mu = np.asarray(mu, dtype=np.float32)
    sigma = np.asarray(sigma, dtype=np.float32)
    amp = np.asarray(amp, dtype=np.float32)
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        inv_s2 = np.float32(1.0) / (sigma * sigma)   # FP32: a scale whose 1/sigma^2 overflows is invalid
    ok = (np.isfinite(mu).all(axis=0) & np.isfinite(sigma) & (sigma > 0) & np.isfinite(amp).all(axis=0)
          & np.isfinite(inv_s2))
    return mu, sigma, amp, ok


def support_mask_f32(px, py, mux, muy, support):
    """The strict support test |x - mu| < D, taken in FP32 one operation at a time."""
    f32 = np.float32
    dx = np.asarray(px, dtype=f32) - f32(mux)
    dy = np.asarray(py, dtype=f32) - f32(muy)
    d2 = dx * dx + dy * dy
    return d2 < f32(support) * f32(support)


def _window(mux, muy, support, width, height):
    """Pixel columns and rows whose centres can lie within the support of one particle."""
    x0 = max(0, int(math.floor(float(mux) - float(support))) - 1)
    x1 = min(width - 1, int(math.ceil(float(mux) + float(support))) + 1)
    y0 = max(0, int(math.floor(float(muy) - float(support))) - 1)
    y1 = min(height - 1, int(math.ceil(float(muy) + float(support))) + 1)
    return x0, x1, y0, y1


def _particle_footprint(k, mu, sigma, support, width, height):
    """(rows, cols, FP64 dx, dy, kernel value) of the pixels in particle k's support."""
    x0, x1, y0, y1 = _window(mu[0, k], mu[1, k], support, width, height)
    if x1 < x0 or y1 < y0:
        return None
    cols = np.arange(x0, x1 + 1)
    rows = np.arange(y0, y1 + 1)
    px = (cols.astype(np.float32) + np.float32(0.5))[None, :]
    py = (rows.astype(np.float32) + np.float32(0.5))[:, None]
    inside = support_mask_f32(px, py, mu[0, k], mu[1, k], support)
    if not inside.any():
        return None
    dx = px.astype(np.float64) - float(mu[0, k])
    dy = py.astype(np.float64) - float(mu[1, k])
    s = float(sigma[k])
    g = np.exp(-(dx * dx + dy * dy) / (s * s)) * inside
    return rows, cols, dx, dy, g


def render_field64(mu, sigma, amp, width, height, support):
    """The image [3][H][W] of the kernel sum (FP64), particles added in index order."""
    mu, sigma, amp, ok = _valid(mu, sigma, amp)
    img = np.zeros((CHANNELS, height, width), dtype=np.float64)
    for k in np.nonzero(ok)[0]:
        fp = _particle_footprint(k, mu, sigma, support, width, height)
        if fp is None:
            continue
        rows, cols, _, _, g = fp
        for c in range(CHANNELS):
            img[c, rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1] += float(amp[c, k]) * g
    return img


def field_grads64(mu, sigma, amp, width, height, support, dL_dimage):
    """(dL/dmu [2][K], dL/dsigma [K], dL/dA [3][K]) in FP64 for upstream dL/dimage [3][H][W]."""
    mu, sigma, amp, ok = _valid(mu, sigma, amp)
    w = np.asarray(dL_dimage, dtype=np.float64)
    K = sigma.shape[0]
    gmu = np.zeros((2, K))
    gsig = np.zeros(K)
    gamp = np.zeros((CHANNELS, K))
    for k in np.nonzero(ok)[0]:
        fp = _particle_footprint(k, mu, sigma, support, width, height)
        if fp is None:
            continue
        rows, cols, dx, dy, g = fp
        wk = w[:, rows[0]:rows[-1] + 1, cols[0]:cols[-1] + 1]
        for c in range(CHANNELS):
            gamp[c, k] = float((wk[c] * g).sum())
        s = float(sigma[k])
        t = sum(wk[c] * float(amp[c, k]) for c in range(CHANNELS)) * g   # dL/dg per pixel
        gmu[0, k] = float((t * 2.0 * dx).sum()) / (s * s)
        gmu[1, k] = float((t * 2.0 * dy).sum()) / (s * s)
        gsig[k] = float((t * 2.0 * (dx * dx + dy * dy)).sum()) / (s * s * s)
    return gmu, gsig, gamp


def l1_loss64(image, target):
    """Mean absolute difference over channels and pixels, and its gradient (sign(0) = 0)."""
    d = np.asarray(image, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.abs(d).mean()), np.sign(d) / d.size


def field_footprints_f32(mu, sigma, amp, width, height, support):
    """The binning view of the particles for the shared tile sort: every particle is a
    disk of radius D around mu (z = 1 for all, so the stable sort keeps particle order
    inside each tile); invalid particles get radius 0 (no tiles)."""
    mu, sigma, amp, ok = _valid(mu, sigma, amp)
    K = sigma.shape[0]
    r = np.where(ok, np.float32(support), np.float32(0.0)).astype(np.float32)
    return {"u": mu[0].copy(), "v": mu[1].copy(), "z": np.ones(K, np.float32), "r": r,
            "width": width, "height": height}
