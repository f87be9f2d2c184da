"""GPU parity of the SSIM term of the loss against the FP64 oracle (oracle/ssim64.py).

Both sides read the same FP32 images. Tolerances follow from FP32 window sums of values
in [0, 1]: the mean SSIM within 1e-5, the gradient within 1e-3 |g| + 1e-3 max|g| (the
derivative maps divide by B1 B2 >= C1 C2, which amplifies FP32 rounding where an image
is locally flat and dark).
"""
import sys

import numpy as np
import pytest

from oracle import ssim64 as Q
import scenegen as S

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible device"
    return torch


@pytest.fixture(scope="module")
def P(torch_cuda):
    import paper_2403_14244_amd as P   # fails loudly if libisogs.so is missing
    return P


def _pair(name):
    rng = np.random.default_rng(7)
    if name == "noise_ragged":
        x = rng.uniform(0, 1, (3, 37, 53))
        y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, 1)
    elif name == "tiny_planes":
        x = rng.uniform(0, 1, (5, 7, 9))
        y = rng.uniform(0, 1, (5, 7, 9))
    elif name == "flat_dark":
        x = np.full((1, 40, 40), 0.02) + rng.normal(0, 1e-3, (1, 40, 40))
        y = np.full((1, 40, 40), 0.05)
    else:   # target512: the 2D fit's target against a blurred, shifted copy
        y = S.field2d_target(512, 512).astype(np.float64)
        x = np.clip(0.8 * np.roll(y, 3, axis=2) + 0.1, 0, 1)
    return x.astype(np.float32), y.astype(np.float32)


CASES = ["noise_ragged", "tiny_planes", "flat_dark", "target512"]


@pytest.mark.parametrize("case", CASES)
def test_ssim_and_gradient_match_oracle(P, torch_cuda, case):
    torch = torch_cuda
    x, y = _pair(case)
    note(f"ssim {case}: {x.shape}")
    ref = Q.ssim64(x, y)
    gref = Q.ssim_grad64(x, y)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    yt = torch.from_numpy(y).cuda()
    s = P.ssim(xt, yt)
    s.backward()
    got = float(s)
    g = xt.grad.cpu().numpy().astype(np.float64)
    note(f"  ssim {got:.7f} vs {ref:.7f}; grad max|d| {np.abs(g - gref).max():.2e} (max|g| {np.abs(gref).max():.2e})")
    assert abs(got - ref) <= 1e-5
    tol = 1e-3 * np.abs(gref) + 1e-3 * np.abs(gref).max()
    assert np.all(np.abs(g - gref) <= tol)


@pytest.mark.parametrize("case", ["noise_ragged", "tiny_planes", "target512"])
def test_loss_matches_oracle_and_is_deterministic(P, torch_cuda, case):
    """The paper's combined loss, value and gradient formed in the library (one forward
    call, one fused gradient kernel): against the FP64 oracle, bitwise repeatable, and
    with lambda = 0 the L1 term's gradient exactly."""
    torch = torch_cuda
    x, y = _pair(case)
    note(f"l1 + ssim loss {case}: {x.shape}")
    lref, gref = Q.l1_ssim_loss64(x, y)
    outs = []
    for _ in range(2):
        xt = torch.from_numpy(x).cuda().requires_grad_(True)
        loss = P.l1_ssim_loss(xt, torch.from_numpy(y).cuda())
        loss.backward()
        outs.append((float(loss), xt.grad.cpu().numpy()))
    assert abs(outs[0][0] - lref) <= 1e-5
    assert outs[0][0] == outs[1][0] and np.array_equal(outs[0][1], outs[1][1])
    tol = 1e-3 * np.abs(gref) + 1e-3 * np.abs(gref).max()
    assert np.all(np.abs(outs[0][1] - gref) <= tol)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    P.l1_ssim_loss(xt, torch.from_numpy(y).cuda(), lam=0.0).backward()
    d = x.astype(np.float64) - y.astype(np.float64)
    np.testing.assert_array_equal(xt.grad.cpu().numpy(), (np.sign(d) * np.float32(1.0 / d.size)).astype(np.float32))


@pytest.mark.parametrize("n_shape", [(3, 1080, 1920), (1, 1, 4097), (2, 3, 5)])
def test_l1_matches_oracle(P, torch_cuda, n_shape):
    # the L1 term: mean |x - y| to FP32 rounding of the per-lane sums, gradient
    # sign(x - y) / n exactly (sign(0) = 0 where clipping made the values equal)
    from oracle import field2d64 as F
    torch = torch_cuda
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, n_shape).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.3, n_shape), 0, 1).astype(np.float32)
    note(f"l1 {n_shape}")
    ref, gref = F.l1_loss64(x, y)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    loss = P.l1_loss(xt, torch.from_numpy(y).cuda())
    (loss * 2.0).backward()
    assert abs(float(loss) - ref) <= 1e-6 * max(1.0, ref)
    np.testing.assert_array_equal(xt.grad.cpu().numpy(), (2.0 * gref).astype(np.float32))
