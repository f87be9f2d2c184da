"""GPU parity of the quadtree initialisation, prune and split of 2D particles against the
FP64 oracle (oracle/tree2d64.py).

The tree's decisions compare an FP64 colour variance with tau on both sides; the sums
are formed in different orders, so every case checks first that no visited cell's
variance lies within 1e-9 of tau (none is flagged), and then requires the same leaves:
count, centres and scales exactly, amplitudes within 1e-6 (FP64 means rounded to FP32).
Prune and split are copies and one FP32 rounding each: bit-exact.
"""
import sys

import numpy as np
import pytest

from oracle import tree2d64 as T
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


def _tree_case(name):
    """(target [3][H][W] FP32, K, root, min_side, tau)"""
    if name == "target512":
        return S.field2d_target(512, 512), 2000, 64, 2, 1e-3
    if name == "target512_budget":
        return S.field2d_target(512, 512), 200, 64, 2, 1e-3
    if name == "ragged_noise":
        rng = np.random.default_rng(3)
        img = S.field2d_target(100, 70, seed=8)
        img = np.clip(img + rng.normal(0, 0.05, img.shape), 0, 1).astype(np.float32)
        return img, 5000, 32, 2, 0.004
    if name == "flat":
        img = np.empty((3, 48, 80), np.float32)
        img[:] = np.float32([0.1, 0.5, 0.9])[:, None, None]
        return img, 100, 16, 1, 1e-6
    raise KeyError(name)


@pytest.mark.parametrize("case", ["target512", "target512_budget", "ragged_noise", "flat"])
def test_tree_init_matches_oracle(P, torch_cuda, case):
    img, K, root, min_side, tau = _tree_case(case)
    note(f"tree init {case}: {img.shape} K={K} root={root} min_side={min_side} tau={tau}")
    (mu, s, a), seen = T.quadtree_init64(img, K, root, min_side, tau, return_stats=True)
    margin = min(abs(v - tau) for lv in seen for v in lv)
    assert margin > 1e-9, "a cell's variance is too close to tau for an exact comparison"
    gm, gs, ga = P.tree_init(torch_cuda.from_numpy(img).cuda(), K, root, min_side, tau)
    note(f"  {s.shape[0]} particles (oracle), {gs.shape[0]} (GPU)")
    assert gs.shape[0] == s.shape[0] <= K
    np.testing.assert_array_equal(gm.cpu().numpy(), mu)
    np.testing.assert_array_equal(gs.cpu().numpy(), s)
    np.testing.assert_allclose(ga.cpu().numpy(), a, rtol=0, atol=1e-6)


def _particles(n=700, seed=4):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0, 100, (2, n)).astype(np.float32)
    s = rng.uniform(0.2, 6.0, n).astype(np.float32)
    a = rng.uniform(-0.2, 0.2, (3, n)).astype(np.float32)
    s[::13] = 0.0
    mu[1, 5::29] = np.nan
    a[2, 7::31] = -np.inf
    return mu, s, a


@pytest.mark.parametrize("thr", [0.0, 0.05, 0.19, 1.0])
def test_prune_matches_oracle(P, torch_cuda, thr):
    mu, s, a = _particles()
    note(f"prune amp_min={thr}")
    om, os_, oa = T.prune64(mu, s, a, thr)
    t = lambda x: torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda()
    gm, gs, ga = P.prune(t(mu), t(s), t(a), thr)
    np.testing.assert_array_equal(gm.cpu().numpy(), om)
    np.testing.assert_array_equal(gs.cpu().numpy(), os_)
    np.testing.assert_array_equal(ga.cpu().numpy(), oa)


@pytest.mark.parametrize("thr", [0.0, 2.5, 100.0])
def test_split_matches_oracle(P, torch_cuda, thr):
    mu, s, a = _particles(seed=6)
    s = np.abs(np.nan_to_num(s, nan=1.0)).astype(np.float32)
    mu = np.nan_to_num(mu, nan=3.0).astype(np.float32)
    note(f"split sigma_max={thr}")
    om, os_, oa = T.split64(mu, s, a, thr)
    t = lambda x: torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda()
    gm, gs, ga = P.split(t(mu), t(s), t(a), thr)
    np.testing.assert_array_equal(gm.cpu().numpy(), om)
    np.testing.assert_array_equal(gs.cpu().numpy(), os_)
    np.testing.assert_array_equal(ga.cpu().numpy(), oa)


def test_empty_inputs(P, torch_cuda):
    e = lambda *sh: torch_cuda.zeros(sh, dtype=torch_cuda.float32, device="cuda")
    for fn, thr in ((P.prune, 0.1), (P.split, 1.0)):
        gm, gs, ga = fn(e(2, 0), e(0), e(3, 0), thr)
        assert gs.shape[0] == 0
