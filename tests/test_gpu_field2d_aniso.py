"""GPU parity of the anisotropic 2D kernel sum (the variant the paper's Table 2 times
against the isotropic one) against the FP64 oracle (oracle/field2d_aniso64.py), through
the C ABI.

Binning is integer work on the same disks of radius D as the isotropic field: bit-exact.
The footprint record copies the centre and amplitudes bit for bit; the conic entries are
FP64 expressions of FP32 parameters rounded once, where the device's cos/sin may differ
from the host's in the last FP64 place, so they are held to one FP32 ulp. Images: the
exponent is a sum of three FP32 products of magnitude up to (s_max/s_min)^2 times the
exponent itself; with the scale ratios below (at most e) the image error stays under
2e-4 max(1, max|img|). Gradients: |d| <= 2e-3 |g| + 2e-4 max|g| per group (theta's
gradient is a difference of the two axes' terms).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from oracle import field2d_aniso64 as FA
from oracle import field2d64 as F
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


def _case(name):
    """(mu [2][K], theta [K], scale [2][K], amp [3][K], width, height, D) in FP32."""
    if name.startswith("fit512"):
        D = 15.0 if name == "fit512_d15" else 50.0
        tgt = S.field2d_target(512, 512)
        mu, s, a = S.field2d_init(tgt, 2000)
        rng = np.random.default_rng(7)
        theta = rng.uniform(-math.pi, math.pi, 2000)
        scale = s[None, :] * np.exp(rng.uniform(-0.5, 0.5, (2, 2000)))
        return mu, theta.astype(np.float32), scale.astype(np.float32), a, 512, 512, D
    rng = np.random.default_rng({"random_ragged": 11, "invalid_and_offimage": 12, "dense_long_lists": 13}[name])
    if name == "random_ragged":
        K, W, H, D = 300, 100, 70, 6.0
        mu = np.stack([rng.uniform(0, W, K), rng.uniform(0, H, K)])
        scale = rng.uniform(0.5, 3.0, (2, K))
        a = rng.uniform(-1, 1, (3, K))
    elif name == "invalid_and_offimage":
        K, W, H, D = 200, 67, 45, 9.5
        mu = np.stack([rng.uniform(-20, W + 20, K), rng.uniform(-20, H + 20, K)])
        scale = rng.uniform(0.4, 4.0, (2, K))
        a = rng.uniform(0, 1, (3, K))
        scale[0, ::17] = 0.0
        scale[1, 5::23] = -1.0
        mu[0, 7::29] = np.nan
        a[1, 11::31] = np.inf
        scale[:, 13] = 1e-30     # the conic overflows in FP32: culled on both sides
    else:   # dense_long_lists: thousands of entries per tile, several staging batches
        K, W, H, D = 3000, 48, 40, 20.0
        mu = np.stack([rng.uniform(10, 38, K), rng.uniform(10, 30, K)])
        scale = rng.uniform(1.0, 6.0, (2, K))
        a = rng.uniform(0, 0.1, (3, K))
    # scale ratio at most e (the bound the image tolerance assumes)
    scale[1] = np.clip(scale[1], scale[0] / math.e, scale[0] * math.e)
    theta = rng.uniform(-math.pi, math.pi, K)
    if name == "invalid_and_offimage":
        theta[19] = np.inf
        scale[1, 5::23] = -1.0
        scale[0, ::17] = 0.0
    return (mu.astype(np.float32), theta.astype(np.float32), scale.astype(np.float32), a.astype(np.float32),
            W, H, D)


CASES = ["random_ragged", "invalid_and_offimage", "dense_long_lists", "fit512_d15", "fit512_d50"]


def _upload(torch, *xs):
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs)


@pytest.mark.parametrize("case", CASES)
def test_field2d_aniso_bins_and_records(P, torch_cuda, case):
    mu, th, sc, a, W, H, D = _case(case)
    note(f"field2d aniso bins {case}: K={th.shape[0]} {W}x{H} D={D}")
    ob = O.bin_sort_ref([FA.field_aniso_footprints_f32(mu, th, sc, a, W, H, D)])
    R = P.Field2DAnisoRenderer(W, H, D)
    fp, conic_c, bins = R.bin(*_upload(torch_cuda, mu, th, sc, a))
    cnt = bins.n_entries()
    assert cnt == ob.keys.shape[0]
    np.testing.assert_array_equal(bins.pidx[:cnt].cpu().numpy().view(np.uint32), ob.pidx)
    np.testing.assert_array_equal(bins.ranges.cpu().numpy().view(np.uint32), ob.ranges)
    np.testing.assert_array_equal(bins.offsets.cpu().numpy().view(np.uint32), ob.offsets)
    np.testing.assert_array_equal(fp.tile_count.cpu().numpy().view(np.uint32), ob.tile_count)
    rec = fp.record.cpu().numpy()
    pc = conic_c.cpu().numpy()
    ok = ob.tile_count > 0
    np.testing.assert_array_equal(rec[ok, 0], mu[0, ok])
    np.testing.assert_array_equal(rec[ok, 1], mu[1, ok])
    np.testing.assert_array_equal(rec[ok, 4:7], a[:, ok].T)
    assert np.all(rec[ok, 7] == np.float32(D))
    P64 = FA.conic(th, sc)[:, ok]
    P32 = P64.astype(np.float32)
    big = np.maximum(np.abs(P32[0]), np.abs(P32[2]))
    ulp = np.spacing(big)
    for got, ref in ((rec[ok, 2], P32[0]), (rec[ok, 3], P32[1]), (pc[ok], P32[2])):
        assert np.all(np.abs(got.astype(np.float64) - ref.astype(np.float64)) <= ulp)
    # invalid particles: all-zero record and conic, no tiles
    valid = FA._valid(mu, th, sc, a)[-1]
    assert np.all(rec[~valid] == 0.0) and np.all(pc[~valid] == 0.0)
    assert np.all(fp.tile_count.cpu().numpy()[~valid] == 0)


@pytest.mark.parametrize("case", CASES)
def test_field2d_aniso_image_matches_oracle(P, torch_cuda, case):
    mu, th, sc, a, W, H, D = _case(case)
    note(f"field2d aniso image {case}: K={th.shape[0]} {W}x{H} D={D}")
    ref = FA.render_field_aniso64(mu, th, sc, a, W, H, D)
    R = P.Field2DAnisoRenderer(W, H, D)
    fp, conic_c, bins = R.bin(*_upload(torch_cuda, mu, th, sc, a))
    img = R.render(fp, conic_c, bins, th.shape[0]).cpu().numpy().astype(np.float64)
    err = np.abs(img - ref).max()
    note(f"  max|d| {err:.2e}, max|img| {np.abs(ref).max():.3f}")
    assert err <= 2e-4 * max(1.0, np.abs(ref).max())
    assert np.all(img[ref == 0.0] == 0.0)


@pytest.mark.parametrize("case", CASES)
def test_field2d_aniso_grads_match_oracle(P, torch_cuda, case):
    mu, th, sc, a, W, H, D = _case(case)
    note(f"field2d aniso grads {case}: K={th.shape[0]} {W}x{H} D={D}")
    if case.startswith("fit512"):
        # the upstream gradient of an L1 fit at these particles
        _, w = F.l1_loss64(FA.render_field_aniso64(mu, th, sc, a, W, H, D), S.field2d_target(512, 512))
    else:
        w = np.random.default_rng(19).normal(size=(3, H, W))
    w = w.astype(np.float32)
    ref = FA.field_aniso_grads64(mu, th, sc, a, W, H, D, w.astype(np.float64))
    R = P.Field2DAnisoRenderer(W, H, D)
    args = _upload(torch_cuda, mu, th, sc, a)
    fp, conic_c, bins = R.bin(*args)
    out = R.grads(*args, fp, conic_c, bins, torch_cuda.from_numpy(w).cuda())
    untouched = fp.tile_count.cpu().numpy() == 0
    for name, got, r in zip(("mu", "theta", "scale", "amp"), out, ref):
        got = got.cpu().numpy().astype(np.float64)
        tol = 2e-3 * np.abs(r) + 2e-4 * np.abs(r).max()
        bad = np.abs(got - r) > tol
        note(f"  d{name}: max|d| {np.abs(got - r).max():.2e} (max|g| {np.abs(r).max():.2e}), "
             f"{int(bad.sum())} over tolerance")
        assert not bad.any()
        assert np.all(got[..., untouched] == 0.0)


def test_field2d_aniso_equal_scales_is_the_isotropic_field(P, torch_cuda):
    """With s1 = s2 = sigma the anisotropic path renders the isotropic image (for any
    angle) and its scale gradients add up to the isotropic sigma gradient."""
    torch = torch_cuda
    W, H, D = 512, 512, 15.0
    tgt = S.field2d_target(512, 512)
    mu, s, a = S.field2d_init(tgt, 2000)
    th = np.random.default_rng(3).uniform(-3, 3, 2000).astype(np.float32)
    sc = np.stack([s, s])
    note("field2d aniso vs iso: K=2000 512x512 D=15")
    Ri, Ra = P.Field2DRenderer(W, H, D), P.Field2DAnisoRenderer(W, H, D)
    mu_t, s_t, a_t = _upload(torch, mu, s, a)
    th_t, sc_t = _upload(torch, th, sc)
    fpi, bi = Ri.bin(mu_t, s_t, a_t)
    fpa, cc, ba = Ra.bin(mu_t, th_t, sc_t, a_t)
    ii = Ri.render(fpi, bi, 2000).cpu().numpy()
    ia = Ra.render(fpa, cc, ba, 2000).cpu().numpy()
    assert np.abs(ii - ia).max() <= 1e-4 * max(1.0, np.abs(ii).max())
    w = torch.from_numpy(np.random.default_rng(4).normal(size=(3, H, W)).astype(np.float32)).cuda()
    gi = [g.cpu().numpy().astype(np.float64) for g in Ri.grads(fpi, bi, 2000, w)]
    ga = [g.cpu().numpy().astype(np.float64) for g in Ra.grads(mu_t, th_t, sc_t, a_t, fpa, cc, ba, w)]
    for got, ref in ((ga[0], gi[0]), (ga[2].sum(axis=0), gi[1]), (ga[3], gi[2])):
        assert np.all(np.abs(got - ref) <= 2e-3 * np.abs(ref) + 2e-4 * np.abs(ref).max())


def test_field2d_aniso_fit_step_decreases_loss_and_is_deterministic(P, torch_cuda):
    torch = torch_cuda
    tgt_np = S.field2d_target(256, 256, seed=4)
    mu0, s0, a0 = S.field2d_init(tgt_np, 600, seed=5)
    th0 = np.zeros(600, np.float32)
    sc0 = np.stack([s0, s0])
    tgt = torch.from_numpy(tgt_np).cuda()
    note("field2d aniso fit: 30 Adam steps, K=600, 256x256, D=15")

    def run():
        mu, th, sc, a = (torch.from_numpy(x.copy()).cuda().requires_grad_(True) for x in (mu0, th0, sc0, a0))
        R = P.Field2DAnisoRenderer(256, 256, 15.0)
        opt = torch.optim.Adam([mu, th, sc, a], lr=0.02)
        losses = []
        for _ in range(30):
            opt.zero_grad()
            img = P.Field2DAnisoRender.apply(mu, th, sc, a, R)
            loss = (img - tgt).abs().mean()
            loss.backward()
            opt.step()
            with torch.no_grad():
                sc.clamp_(min=0.3)
            losses.append(float(loss))
        return losses, img.detach().cpu().numpy()

    l1, img1 = run()
    l2, img2 = run()
    assert l1[-1] < 0.8 * l1[0]
    assert l1 == l2 and np.array_equal(img1, img2)
