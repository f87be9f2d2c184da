"""GPU parity of the 2D kernel-sum representation (Section 3) against the FP64 oracle.

Both sides read the same FP32 parameters. Binning is integer work and must be bit-exact
(including the footprint records, which are copies or one correctly rounded division);
images must match to max-abs 1e-4 (the support decision is taken in FP32 on both sides,
so no pixel is flagged); gradients to |d| <= 1e-3 |g| + 1e-4 max|g| per group.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import field2d64 as F
import scenegen as S

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


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


def _case(name):
    """(mu [2][K], sigma [K], amp [3][K], width, height, D) in FP32."""
    if name.startswith("fit512"):
        D = 15.0 if name == "fit512_d15" else 50.0
        tgt = S.field2d_target(512, 512)
        mu, s, a = S.field2d_init(tgt, 2000)
        return mu, s, a, 512, 512, D
    rng = np.random.default_rng({"random_ragged": 1, "invalid_and_offimage": 2, "dense_long_lists": 3}[name])
    if name == "random_ragged":
        K, W, H, D = 300, 100, 70, 6.0
        mu = np.stack([rng.uniform(0, W, K), rng.uniform(0, H, K)])
        s = rng.uniform(0.5, 3.0, K)
        a = rng.uniform(-1, 1, (3, K))
    elif name == "invalid_and_offimage":
        K, W, H, D = 200, 67, 45, 9.5
        mu = np.stack([rng.uniform(-20, W + 20, K), rng.uniform(-20, H + 20, K)])
        s = rng.uniform(0.3, 4.0, K)
        a = rng.uniform(0, 1, (3, K))
        s[::17] = 0.0
        s[5::23] = -1.0
        mu[0, 7::29] = np.nan
        a[1, 11::31] = np.inf
        s[13] = 1e-30        # 1/sigma^2 overflows in FP32: culled on both sides
    else:   # dense_long_lists: thousands of entries per tile, several staging batches
        K, W, H, D = 3000, 48, 40, 20.0
        mu = np.stack([rng.uniform(10, 38, K), rng.uniform(10, 30, K)])
        s = rng.uniform(1.0, 6.0, K)
        a = rng.uniform(0, 0.1, (3, K))
    return mu.astype(np.float32), s.astype(np.float32), a.astype(np.float32), W, H, D


CASES = ["random_ragged", "invalid_and_offimage", "dense_long_lists", "fit512_d15", "fit512_d50"]


def _upload(torch, mu, s, a):
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t(mu), t(s), t(a)


@pytest.mark.parametrize("case", CASES)
def test_field2d_bins_bit_exact(P, torch_cuda, case):
    mu, s, a, W, H, D = _case(case)
    note(f"field2d bins {case}: K={s.shape[0]} {W}x{H} D={D}")
    ob = O.bin_sort_ref([F.field_footprints_f32(mu, s, a, W, H, D)])
    R = P.Field2DRenderer(W, H, D)
    fp, bins = R.bin(*_upload(torch_cuda, mu, s, a))
    cnt = bins.n_entries()
    assert cnt == ob.keys.shape[0]
    np.testing.assert_array_equal(bins.pidx[:cnt].cpu().numpy().view(np.uint32), ob.pidx)
    np.testing.assert_array_equal(bins.ranges.cpu().numpy().view(np.uint32), ob.ranges)
    np.testing.assert_array_equal(bins.offsets.cpu().numpy().view(np.uint32), ob.offsets)
    np.testing.assert_array_equal(fp.tile_count.cpu().numpy().view(np.uint32), ob.tile_count)
    rec = fp.record.cpu().numpy()
    ok = ob.tile_count > 0
    np.testing.assert_array_equal(rec[ok, 0], mu[0, ok])
    np.testing.assert_array_equal(rec[ok, 1], mu[1, ok])
    np.testing.assert_array_equal(rec[ok, 2], np.float32(1.0) / (s[ok] * s[ok]))
    np.testing.assert_array_equal(rec[ok, 4:7], a[:, ok].T)


@pytest.mark.parametrize("case", CASES)
def test_field2d_image_matches_oracle(P, torch_cuda, case):
    mu, s, a, W, H, D = _case(case)
    note(f"field2d image {case}: K={s.shape[0]} {W}x{H} D={D}")
    ref = F.render_field64(mu, s, a, W, H, D)
    R = P.Field2DRenderer(W, H, D)
    fp, bins = R.bin(*_upload(torch_cuda, mu, s, a))
    img = R.render(fp, bins, s.shape[0]).cpu().numpy().astype(np.float64)
    err = np.abs(img - ref).max()
    note(f"  max|d| {err:.2e}, max|img| {np.abs(ref).max():.3f}")
    assert err <= IMG_TOL
    # pixels that no particle's support reaches are exactly zero
    assert np.all(img[ref == 0.0] == 0.0)


@pytest.mark.parametrize("case", CASES)
def test_field2d_grads_match_oracle(P, torch_cuda, case):
    mu, s, a, W, H, D = _case(case)
    note(f"field2d grads {case}: K={s.shape[0]} {W}x{H} D={D}")
    rng = np.random.default_rng(9)
    if case.startswith("fit512"):
        # the upstream gradient of the paper's L1 fit at the initial particles
        _, w = F.l1_loss64(F.render_field64(mu, s, a, W, H, D), S.field2d_target(512, 512))
    else:
        w = rng.normal(size=(3, H, W))
    w = w.astype(np.float32)
    gmu, gs, ga = F.field_grads64(mu, s, a, W, H, D, w.astype(np.float64))
    R = P.Field2DRenderer(W, H, D)
    fp, bins = R.bin(*_upload(torch_cuda, mu, s, a))
    out = R.grads(fp, bins, s.shape[0], torch_cuda.from_numpy(w).cuda())
    untouched = fp.tile_count.cpu().numpy() == 0
    for name, got, ref in zip(("mu", "sigma", "amp"), out, (gmu, gs, ga)):
        got = got.cpu().numpy().astype(np.float64)
        tol = 1e-3 * np.abs(ref) + 1e-4 * np.abs(ref).max()
        bad = np.abs(got - ref) > tol
        note(f"  d{name}: max|d| {np.abs(got - ref).max():.2e} (max|g| {np.abs(ref).max():.2e}), "
             f"{int(bad.sum())} over tolerance")
        assert not bad.any()
        # culled particles and particles whose support misses the image get exact zeros
        assert np.all(got[..., untouched] == 0.0)


def test_field2d_fit_step_decreases_loss_and_is_deterministic(P, torch_cuda):
    torch = torch_cuda
    tgt_np = S.field2d_target(256, 256, seed=4)
    mu0, s0, a0 = S.field2d_init(tgt_np, 600, seed=5)
    tgt = torch.from_numpy(tgt_np).cuda()
    note("field2d fit: 30 Adam steps, K=600, 256x256, D=15")

    def run():
        mu, s, a = (torch.from_numpy(x.copy()).cuda().requires_grad_(True) for x in (mu0, s0, a0))
        R = P.Field2DRenderer(256, 256, 15.0)
        opt = torch.optim.Adam([mu, s, a], lr=0.02)
        losses = []
        for _ in range(30):
            opt.zero_grad()
            img = P.Field2DRender.apply(mu, s, a, R)
            loss = (img - tgt).abs().mean()
            loss.backward()
            opt.step()
            with torch.no_grad():
                s.clamp_(min=0.3)
            losses.append(float(loss))
        return losses, img.detach().cpu().numpy()

    l1, img1 = run()
    l2, img2 = run()
    assert l1[-1] < 0.8 * l1[0]
    assert l1 == l2 and np.array_equal(img1, img2)


def test_field2d_capacity_overflow_recovers(P, torch_cuda):
    mu, s, a, W, H, D = _case("random_ragged")
    note("field2d capacity overflow")
    R = P.Field2DRenderer(W, H, D)
    # far too small: the first binning overflows, the second runs with the exact count
    fp, bins = R.bin(*_upload(torch_cuda, mu, s, a), capacity=16)
    ob = O.bin_sort_ref([F.field_footprints_f32(mu, s, a, W, H, D)])
    assert bins.capacity > ob.keys.shape[0] and bins.n_entries() == ob.keys.shape[0]
    # the default capacity bounds every binning: at most (ceil(2D/16) + 1)^2 tiles a particle
    assert int(ob.tile_count.max()) <= (int(np.ceil(2 * D / 16)) + 1) ** 2 < R.tiles_bound()
    img = R.render(fp, bins, s.shape[0]).cpu().numpy()
    assert np.abs(img - F.render_field64(mu, s, a, W, H, D)).max() <= IMG_TOL


def test_field2d_fit_step_replays_in_a_hip_graph(P, torch_cuda):
    # the whole step (binning, kernel sum, L1 + SSIM loss, gradients, Adam) captured once
    # and replayed: every replay, with eager work and synchronisations in between, must
    # leave the parameters bitwise where the same steps taken eagerly leave them
    torch = torch_cuda
    tgt_np = S.field2d_target(128, 128, seed=6)
    mu0, s0, a0 = S.field2d_init(tgt_np, 300, seed=7)
    tgt = torch.from_numpy(tgt_np).cuda()
    note("field2d fit step in a HIP graph: K=300, 128x128, D=12")

    def make():
        params = [torch.from_numpy(x.copy()).cuda().requires_grad_(True) for x in (mu0, s0, a0)]
        opt = torch.optim.Adam(params, lr=0.02, capturable=True)
        R = P.Field2DRenderer(128, 128, 12.0)

        def step():
            opt.zero_grad(set_to_none=True)
            loss = P.l1_ssim_loss(P.Field2DRender.apply(*params, R), tgt)
            loss.backward()
            opt.step()
            with torch.no_grad():
                params[1].clamp_(min=0.3)
            return loss
        return params, step

    eager_params, eager_step = make()
    graph_params, graph_step = make()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):            # warm-up: workspaces, capacity, optimizer state
            eager_step()
            graph_step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        static_loss = graph_step()
    for i in range(4):
        g.replay()
        eager_loss = eager_step()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        assert float(static_loss) == float(eager_loss), f"replay {i}: loss differs"
        for a, b in zip(graph_params, eager_params):
            assert torch.equal(a, b), f"replay {i}: parameters differ"
