"""FP64 oracle of the SSIM term of the paper's loss (Section 3, the loss equation).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The GPU library never calls
it and shares no code, constants table or helper with it.

The paper writes its loss as (1 - lambda) times the L1 error plus lambda times an SSIM
term, lambda = 0.2, without defining SSIM or the sign of the term (the formula is
garbled). Readings:

* the term is lambda (1 - SSIM), so that the loss decreases as the images agree;
* SSIM is the structural similarity index of Wang, Bovik, Sheikh and Simoncelli (IEEE
  TIP 2004) in its usual form: per channel, local statistics under an 11 x 11 Gaussian
  window of standard deviation 1.5 (normalised to sum 1), stabilisers C1 = (0.01 L)^2
  and C2 = (0.03 L)^2 with dynamic range L = 1,

      S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),

  where mu = G * x, s_x^2 = G * x^2 - mu_x^2, s_xy = G * (x y) - mu_x mu_y, and the image
  outside its borders counts as zero (the window is not renormalised there);
* the reported SSIM is the mean of S over channels and pixels.

Gradient with respect to the rendered image x (the target y is a constant): with
m1 = G*x, m2 = G*y, e11 = G*x^2, e12 = G*(x y), A1 = 2 m1 m2 + C1, A2 = 2 (e12 - m1 m2) + C2,
B1 = m1^2 + m2^2 + C1, B2 = (e11 - m1^2) + (e22 - m2^2) + C2 and N the element count,

    dSSIM/dx = (1/N) [G^T * dS/dm1 + 2 x (G^T * dS/de11) + y (G^T * dS/de12)]
    dS/de11 = -A1 A2 / (B1 B2^2),  dS/de12 = 2 A1 / (B1 B2),
    dS/dm1  = 2 m2 (A2 - A1) / (B1 B2) - 2 m1 A1 A2 / (B1^2 B2) + 2 m1 A1 A2 / (B1 B2^2),

G^T being the transposed (here equal, the window is symmetric) zero-padded filter.

Pins (tests/test_ssim_oracle.py): SSIM(x, x) = 1, symmetry in x and y, the closed form
of two constant images at interior pixels, a brute-force window sum on a tiny image,
and FP64 central differences of the gradient.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import correlate1d

WINDOW = 11
WINDOW_SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA = 0.2


def gaussian_window():
    """The 1D window (length 11, sigma 1.5, sum 1); the 2D window is its outer product."""
    r = np.arange(WINDOW, dtype=np.float64) - (WINDOW - 1) / 2
    g = np.exp(-r * r / (2.0 * WINDOW_SIGMA * WINDOW_SIGMA))
    return g / g.sum()


def blur(a):
    """G * a over the last two axes, zero outside the image (separable correlation)."""
    g = gaussian_window()
    a = np.asarray(a, dtype=np.float64)
    return correlate1d(correlate1d(a, g, axis=-1, mode="constant", cval=0.0), g, axis=-2, mode="constant", cval=0.0)


def _stats(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m1, m2 = blur(x), blur(y)
    e11, e22, e12 = blur(x * x), blur(y * y), blur(x * y)
    A1 = 2.0 * m1 * m2 + C1
    A2 = 2.0 * (e12 - m1 * m2) + C2
    B1 = m1 * m1 + m2 * m2 + C1
    B2 = (e11 - m1 * m1) + (e22 - m2 * m2) + C2
    return x, y, m1, m2, A1, A2, B1, B2


def ssim_map64(x, y):
    """S per channel and pixel, for images [C][H][W]."""
    _, _, _, _, A1, A2, B1, B2 = _stats(x, y)
    return (A1 * A2) / (B1 * B2)


def ssim64(x, y):
    """Mean SSIM over channels and pixels."""
    return float(ssim_map64(x, y).mean())


def ssim_grad64(x, y):
    """dSSIM/dx for the mean SSIM (y constant)."""
    x, y, m1, m2, A1, A2, B1, B2 = _stats(x, y)
    n = x.size
    d_e11 = -A1 * A2 / (B1 * B2 * B2)
    d_e12 = 2.0 * A1 / (B1 * B2)
    d_m1 = (2.0 * m2 * (A2 - A1) / (B1 * B2) - 2.0 * m1 * A1 * A2 / (B1 * B1 * B2)
            + 2.0 * m1 * A1 * A2 / (B1 * B2 * B2))
    return (blur(d_m1) + 2.0 * x * blur(d_e11) + y * blur(d_e12)) / n


def l1_ssim_loss64(x, y, lam=LAMBDA):
    """The paper's loss read as (1 - lambda) mean|x - y| + lambda (1 - SSIM(x, y)), and its
    gradient with respect to x (sign(0) = 0 for the L1 part)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = x - y
    loss = (1.0 - lam) * float(np.abs(d).mean()) + lam * (1.0 - ssim64(x, y))
    grad = (1.0 - lam) * np.sign(d) / d.size - lam * ssim_grad64(x, y)
    return loss, grad
