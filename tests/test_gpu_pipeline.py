"""GPU parity of every stage of the rasterizer against the FP64 oracle, through the C ABI.

Stage tests give both sides identical FP32 inputs produced by the oracle, so:
  * binning and sorting must be bit-exact (integer work);
  * compositing must match to max-abs 1e-4 on every pixel whose FP64 walk does not pass
    within rounding of a discrete decision (alpha = 1/255, T = 1e-4); such pixels are
    flagged, must be rare, and must match one of the results the oracle gets by taking
    each in-band decision both ways, to the same 1e-4;
  * gradients must match to 1e-3 |g| + 1e-4 max|g| for every parameter; the upstream
    gradient gives no weight to flagged pixels, where the two sides may legitimately
    walk different entries;
  * projection must match the FP64 values to within FP32 rounding.
End-to-end tests (GPU footprints from the particle parameters) widen the flag bands by
what the footprints' own FP32 rounding can change (oracle.footprint_uncertainty).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import scenegen as S
from tests import _helpers as TH

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


def ulp32(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


def small_mix(n=20_000, seed=3, deg=3):
    return S.mixture_scene(n, seed=seed, log_scale_mean=math.log(0.012), sh_degree=deg)


PROJECT_CASES = {
    "cube10k_256": lambda: ([S.workload_scene("cube10k_256")], S.workload_cameras("cube10k_256")),
    "mix20k_deg3_321x203": lambda: ([small_mix()], [S.orbit_camera(0.7, 4.0, 321, 203)]),
    "mix20k_deg1_1920x1080": lambda: ([small_mix(deg=1)], [S.orbit_camera(1.3, 4.0, 1920, 1080)]),
    "batch_mixed": lambda: ([S.workload_scene("cube10k_256"), small_mix(5000, 4, 2)],
                            [S.workload_cameras("cube10k_256")[0], S.orbit_camera(2.0, 3.5, 100, 60)]),
}


@pytest.mark.parametrize("case", list(PROJECT_CASES))
def test_project_matches_oracle(P, torch_cuda, case):
    note(f"project {case}")
    scenes, cams = PROJECT_CASES[case]()
    R = P.Rasterizer()
    fp = R.project([P.GaussianScene.from_host(s) for s in scenes], cams)
    torch_cuda.cuda.synchronize()
    foot = fp.record[:, :4].cpu().numpy()
    colr = fp.record[:, 4:].cpu().numpy()
    z = fp.depth.cpu().numpy()
    tc = fp.tile_count.cpu().numpy()
    projs = [O.project64(s, c) for s, c in zip(scenes, cams)]
    views = TH.oracle_f32_footprints(projs, cams)
    ob = O.bin_sort_ref(O.f32_views(projs, cams))
    off = 0
    for pr, vw in zip(projs, views):
        n = pr.u.shape[0]
        sl = slice(off, off + n)
        vis = pr.visible
        assert ((foot[sl, 3] > 0) == vis).all()
        assert vis.sum() > 0.3 * n
        # u, v: FP64 computation rounded once -> within half an FP32 ulp of the FP64 value,
        # the bound the end-to-end comparisons assume (oracle.footprint_uncertainty)
        pe, _ = O.footprint_uncertainty(pr)
        for k, arr, ref in (("u", foot[sl, 0], pr.u), ("v", foot[sl, 1], pr.v)):
            d = np.abs(arr[vis].astype(np.float64) - ref[vis])
            assert (d <= pe[vis]).all(), (k, float((d / pe[vis]).max()))
        # z: within one ulp of the oracle's FP32 depth (the order the comparisons allow for)
        d = np.abs(z[sl][vis].astype(np.float64) - vw["z"][vis].astype(np.float64))
        assert (d <= ulp32(vw["z"][vis])).all(), ("z", d.max())
        np.testing.assert_allclose(foot[sl, 2][vis], vw["is2"][vis], rtol=2 ** -21)
        np.testing.assert_array_equal(foot[sl, 3][vis], vw["o"][vis])
        np.testing.assert_allclose(colr[sl, :3][vis].T, vw["rgb"][:, vis], atol=1e-5)
        np.testing.assert_allclose(colr[sl, 3][vis], vw["r"][vis], rtol=2 ** -21)
        # tile counts: identical wherever the FP32 footprint is bit-identical
        same = ((foot[sl, 0] == vw["u"]) & (foot[sl, 1] == vw["v"]) & (colr[sl, 3] == vw["r"]))
        assert same[vis].mean() > 0.99
        np.testing.assert_array_equal(tc[sl][same], ob.tile_count[sl][same].astype(np.int64))
        off += n


def _bin_case(name):
    if name == "cube10k_256":
        sc, cams = [S.workload_scene("cube10k_256")], S.workload_cameras("cube10k_256")
        projs = [O.project64(s, c) for s, c in zip(sc, cams)]
        return TH.oracle_f32_footprints(projs, cams), cams
    if name == "mix_batch_3views":
        sc = small_mix(30_000, 5, 3)
        cams = [S.orbit_camera(0.3 * i, 4.0, w, h) for i, (w, h) in enumerate([(256, 256), (333, 190), (64, 48)])]
        projs = [O.project64(sc, c) for c in cams]
        return TH.oracle_f32_footprints(projs, cams), cams
    if name in ("random_ties", "random_wide"):
        ties = name == "random_ties"
        views, cams = [], []
        for k, (w, h) in enumerate([(200, 120), (47, 33)]):
            u, v, z, r = S.random_projected(3000, w, h, seed=20 + k, max_radius=40.0 if not ties else 10.0,
                                            depth_ties=ties)
            views.append(TH.synthetic_f32_footprints(u, v, z, r, w, h, seed=k))
            cams.append(S.look_at_camera((0, 0, 3), width=w, height=h))
        return views, cams
    if name == "mix200k_1080p":
        sc = S.mixture_scene(200_000, seed=7)
        cams = [S.orbit_camera(1.0, 4.0, 1920, 1080)]
        projs = [O.project64(sc, c) for c in cams]
        return TH.oracle_f32_footprints(projs, cams), cams
    if name in ("crowd_wide_depth", "crowd_narrow_depth"):
        # one tile with thousands of entries: the segment sort's multi-chunk path, with an
        # even (wide depths) and an odd (eight tied depth values) number of digit passes
        wide = name == "crowd_wide_depth"
        n = 9000 if wide else 5000
        u, v, z, r = S.crowded_projected(n, 96, 64, 40.0, 24.0, 7.5, seed=31 if wide else 32, max_radius=6.0,
                                         depths=None if wide else [2.0 + k / 8 for k in range(8)])
        return [TH.synthetic_f32_footprints(u, v, z, r, 96, 64, seed=3)], [S.look_at_camera((0, 0, 3), width=96, height=64)]
    if name == "segment_boundaries":
        # footprints inside one tile each, one segment per view at the size limits of the
        # segment sort's paths: 64 (rank by comparison in one wave), 65, 512 (largest
        # sorted by one wave), 513, 1024, 1025, 4096 (largest radix-sorted in LDS by a
        # workgroup), 4097 (through the workspace), 8192 and 8193
        views, cams = [], []
        for k, n in enumerate((64, 65, 512, 513, 1024, 1025, 4096, 4097, 8192, 8193)):
            u, v, z, r = S.crowded_projected(n, 48, 32, 24.0, 8.0, 2.0, seed=40 + k, max_radius=0.5)
            views.append(TH.synthetic_f32_footprints(u, v, z, r, 48, 32, seed=k))
            cams.append(S.look_at_camera((0, 0, 3), width=48, height=32))
        return views, cams
    if name in ("segment_chunked", "segment_chunked_ties"):
        # segments sorted by all workgroups in 4096-entry chunks (longer than 16384 entries):
        # 16384 (the last one sorted by one workgroup), 16385 (a chunk of one entry), 40000;
        # with ties: 70000 entries of 8 depth values (only one byte of the depth bits varies:
        # three passes skipped, the result left in the workspace) and 20000 over [0.5, 80]
        # (all four bytes vary)
        ties = name == "segment_chunked_ties"
        views, cams = [], []
        sizes = ((70000, [2.0 + k / 8 for k in range(8)]), (20000, None)) if ties else \
            ((16384, None), (16385, None), (40000, None))
        for k, (n, dep) in enumerate(sizes):
            u, v, z, r = S.crowded_projected(n, 48, 32, 24.0, 8.0, 2.0, seed=80 + k + 10 * ties, max_radius=0.5,
                                             depths=dep)
            views.append(TH.synthetic_f32_footprints(u, v, z, r, 48, 32, seed=k))
            cams.append(S.look_at_camera((0, 0, 3), width=48, height=32))
        return views, cams
    if name == "tile_edges":
        # disks whose edges fall on, just inside and just outside tile borders and pixel
        # centres (the candidate tile box and the membership test at their margins), in a
        # 200x170 view whose last tile column and row are partial
        offs = np.array([0.0, 0.25, 0.5, 0.5 - 2.0 ** -10, 0.5 + 2.0 ** -10, 8.0, 15.5, 15.75, 16.0 - 2.0 ** -10])
        radii = np.array([0.25, 0.5, 1.0, 4.0, 7.5, 15.5, 16.0, 16.5, 24.0, 40.0])
        us, vs, rs = [], [], []
        for k in (0, 3, 11, 12):
            for ox in offs:
                for oy in offs[::3]:
                    for r in radii:
                        us.append(16 * k + ox)
                        vs.append(16 * (k % 10) + oy)
                        rs.append(r)
        u = np.array(us, np.float32)
        v = np.array(vs, np.float32)
        r = np.array(rs, np.float32)
        z = np.random.default_rng(5).uniform(0.5, 8.0, u.shape[0]).astype(np.float32)
        return [TH.synthetic_f32_footprints(u, v, z, r, 200, 170, seed=9)], [S.look_at_camera((0, 0, 3), width=200, height=170)]
    if name == "segment_groups":
        # segments of 513 .. 4096 entries, one per view, sorted several to a workgroup (up to
        # 1024 entries four at once, up to 2048 two at once): odd numbers in each size class
        # leave groups empty, and tied depths (one digit pass) share workgroups with spread
        # ones (three passes)
        views, cams = [], []
        tied = [2.0 + k / 8 for k in range(8)]
        for k, n in enumerate((513, 600, 700, 1024, 777, 888, 999, 1025, 1500, 2048, 2049, 3000, 4096)):
            u, v, z, r = S.crowded_projected(n, 48, 32, 24.0, 8.0, 2.0, seed=120 + k, max_radius=0.5,
                                             depths=tied if k % 3 == 1 else None)
            views.append(TH.synthetic_f32_footprints(u, v, z, r, 48, 32, seed=k))
            cams.append(S.look_at_camera((0, 0, 3), width=48, height=32))
        return views, cams
    if name == "emit_runs":
        # the emit step writes a chunk of 256 particles' entries through LDS when the chunk
        # holds at most 2048 of them, else each particle writes its own: views of small,
        # medium (chunks on both sides of 2048) and large disks
        rng = np.random.default_rng(91)
        views, cams = [], []
        for k, (n, r0, r1) in enumerate([(1536, 0.5, 12.0), (1280, 10.8, 22.8), (768, 40.0, 90.0)]):
            u = rng.uniform(0, 400, n).astype(np.float32)
            v = rng.uniform(0, 300, n).astype(np.float32)
            z = rng.uniform(0.5, 9.0, n).astype(np.float32)
            r = rng.uniform(r0, r1, n).astype(np.float32)
            views.append(TH.synthetic_f32_footprints(u, v, z, r, 400, 300, seed=k))
            cams.append(S.look_at_camera((0, 0, 3), width=400, height=300))
        return views, cams
    if name == "segment_ties_bucketed":
        # one 3000-entry segment whose depths take 64 values: every bucket of the leading
        # bits holds one value many times, so positions decide the order inside buckets
        u, v, z, r = S.crowded_projected(3000, 48, 32, 24.0, 8.0, 2.0, seed=60, max_radius=0.5,
                                         depths=[1.0 + k / 16 for k in range(64)])
        return [TH.synthetic_f32_footprints(u, v, z, r, 48, 32)], [S.look_at_camera((0, 0, 3), width=48, height=32)]
    if name == "all_tiles_long":
        # every tile of a 208x200 view holds more than 512 entries, so each of the 64 lists
        # of long segments receives two or three tiles (tile ids equal modulo 64)
        rng = np.random.default_rng(70)
        n = 30_000
        u = rng.uniform(0, 208, n).astype(np.float32)
        v = rng.uniform(0, 200, n).astype(np.float32)
        z = rng.uniform(0.5, 9.0, n).astype(np.float32)
        r = rng.uniform(12.0, 20.0, n).astype(np.float32)
        cam = S.look_at_camera((0, 0, 3), width=208, height=200)
        return [TH.synthetic_f32_footprints(u, v, z, r, 208, 200, seed=5)], [cam]
    if name == "single_tile":
        u, v, z, r = S.random_projected(400, 16, 16, seed=50, max_radius=6.0, depth_ties=True)
        return [TH.synthetic_f32_footprints(u, v, z, r, 16, 16)], [S.look_at_camera((0, 0, 3), width=16, height=16)]
    if name == "empty_and_culled":
        sc = small_mix(500, 6, 0)
        sc.pos[2, :] = 50.0     # all behind a camera looking down -z from z=3 ... culled
        cams = [S.look_at_camera((0, 0, 3), width=40, height=40), S.look_at_camera((0, 0, 3), width=16, height=16)]
        projs = [O.project64(sc, cams[0])]
        views = TH.oracle_f32_footprints(projs, cams[:1])
        empty = TH.synthetic_f32_footprints(*(np.zeros(0, np.float32),) * 4, 16, 16)
        return views + [empty], cams
    raise KeyError(name)


BIN_CASES = ["cube10k_256", "mix_batch_3views", "random_ties", "random_wide", "mix200k_1080p", "empty_and_culled",
             "crowd_wide_depth", "crowd_narrow_depth", "segment_boundaries", "segment_groups", "tile_edges", "segment_ties_bucketed", "single_tile",
             "all_tiles_long", "segment_chunked", "segment_chunked_ties", "emit_runs"]


@pytest.mark.parametrize("case", BIN_CASES)
def test_bin_sort_bit_exact(P, torch_cuda, case):
    views, cams = _bin_case(case)
    ob = O.bin_sort_ref(views)
    note(f"bin_sort {case}: {ob.keys.shape[0]} entries")
    if case == "emit_runs":
        # entries per chunk of 256 particles of a view: both sides of 2048 occur
        ends = np.append(ob.offsets[1:].astype(np.int64), ob.keys.shape[0])
        p0, runs = 0, []
        for vw in views:
            n = vw["u"].shape[0]
            runs += [int(ends[min(p0 + c + 255, p0 + n - 1)] - int(ob.offsets[p0 + c])) for c in range(0, n, 256)]
            p0 += n
        assert min(runs) <= 2048 < max(runs) and sum(2000 <= x <= 2048 for x in runs) >= 2 and \
            sum(2048 < x <= 2100 for x in runs) >= 1, runs
    R = P.Rasterizer()
    fp = TH.upload_footprints(views, ob)
    npv = [v["u"].shape[0] for v in views]
    bins = R.bin_sort(fp, npv, cams, with_keys=True)
    torch_cuda.cuda.synchronize()
    cnt = bins.n_entries()
    assert cnt == ob.keys.shape[0]
    np.testing.assert_array_equal(bins.keys[:cnt].cpu().numpy().view(np.uint64), ob.keys)
    np.testing.assert_array_equal(bins.pidx[:cnt].cpu().numpy().view(np.uint32), ob.pidx)
    np.testing.assert_array_equal(bins.ranges.cpu().numpy().view(np.uint32), ob.ranges)
    np.testing.assert_array_equal(bins.offsets.cpu().numpy().view(np.uint32), ob.offsets)
    # without the optional keys the entry order is the same
    nk = R.bin_sort(fp, npv, cams)
    assert nk.keys is None
    np.testing.assert_array_equal(nk.pidx[:cnt].cpu().numpy().view(np.uint32), ob.pidx)
    np.testing.assert_array_equal(nk.ranges.cpu().numpy().view(np.uint32), ob.ranges)


def test_bin_sort_capacity_overflow_reports_and_recovers(P, torch_cuda):
    views, cams = _bin_case("cube10k_256")
    ob = O.bin_sort_ref(views)
    note("bin_sort capacity overflow")
    R = P.Rasterizer()
    fp = TH.upload_footprints(views, ob)
    small = R.bin_sort(fp, [views[0]["u"].shape[0]], cams, check=False, capacity=1000)
    torch_cuda.cuda.synchronize()
    assert int(small.status.item()) == P._abi.ISOGS_ERR_CAPACITY
    assert small.n_entries() == ob.keys.shape[0]
    with pytest.raises(P.IsoGSError):
        small.verify()
    # the render of an overflowed bin set marks every pixel invalid (NaN colour and T,
    # n_last 0), in both the spatial and the longest-first launches
    for out in (R.render_fwd(fp, [views[0]["u"].shape[0]], small, cams),
                R.render_fwd_ordered(fp, [views[0]["u"].shape[0]], small, cams),
                R.render_fwd_ordered(fp, [views[0]["u"].shape[0]], small, cams, wide=True)):
        img, T, nl = out
        assert bool(torch_cuda.isnan(img).all()) and bool(torch_cuda.isnan(T).all()) and int(nl.abs().sum()) == 0
    # growing on demand gives the exact lists
    ok = R.bin_sort(fp, [views[0]["u"].shape[0]], cams, with_keys=True)
    assert ok.capacity >= ob.keys.shape[0]
    np.testing.assert_array_equal(ok.keys[:ok.n_entries()].cpu().numpy().view(np.uint64), ob.keys)




RENDER_CASES = ["cube10k_256", "mix_batch_3views", "dense_termination"]


def _render_case(name):
    if name == "dense_termination":
        sc = S.uniform_cube_scene(6000, seed=9, log_scale_mean=math.log(0.08))
        sc.opacity[:] = np.float32(0.85)
        cams = [S.look_at_camera((0, 0, 3), width=96, height=80)]
        projs = [O.project64(sc, cams[0])]
        return TH.oracle_f32_footprints(projs, cams), cams
    return _bin_case(name)


@pytest.mark.parametrize("case", RENDER_CASES)
def test_render_fwd_matches_oracle(P, torch_cuda, case):
    views, cams = _render_case(case)
    ob = O.bin_sort_ref(views)
    bg = (0.1, 0.3, 0.2)
    note(f"render_fwd {case}: {ob.keys.shape[0]} entries")
    R = P.Rasterizer()
    fp = TH.upload_footprints(views, ob)
    gb = TH.upload_bins(ob)
    img, T, nl = R.render_fwd(fp, [v["u"].shape[0] for v in views], gb, cams, bg)
    torch_cuda.cuda.synchronize()
    gi = TH.split_flat(img.cpu().numpy(), cams)
    gT = TH.split_flat(T.cpu().numpy(), cams, 1)
    gn = TH.split_flat(nl.cpu().numpy(), cams, 1)
    ref = TH.oracle_render_f32(views, ob, bg)
    outs = TH.f32_footprint_outcomes(views, ob, bg)
    for k, (oimg, oT, onl, ofl) in enumerate(ref):
        mx, nfl, mf = TH.check_image(gi[k], gT[k], oimg, oT, ofl, outs[k], what=f"{case} view {k}")
        note(f"  view {k}: max|d| {mx:.2e}, flagged {nfl} (nearest valid outcome within {mf:.2e})")
        np.testing.assert_array_equal(gn[k][~ofl], onl[~ofl])
    if case == "dense_termination":
        assert (ref[0][1] < O.T_MIN).mean() > 0.2


def _e2e_scenes(name):
    if name == "cube10k_256":
        return [S.workload_scene("cube10k_256")], S.workload_cameras("cube10k_256")
    if name == "mix50k_deg3_480x270":
        sc = S.mixture_scene(50_000, seed=2, log_scale_mean=math.log(0.008))
        return [sc, sc], [S.orbit_camera(0.5, 4.0, 480, 270), S.orbit_camera(2.5, 4.0, 480, 270)]
    raise KeyError(name)


def check_end_to_end(scenes, cams, imgs, T, bg=(0.0, 0.0, 0.0), what="", max_flag_frac=0.01):
    """GPU images (list of [3, H, W]) and packed T_final against the oracle's end-to-end
    render, flags widened by the footprints' FP32 rounding. Returns the oracle's flags."""
    ores = O.render_views(scenes, cams, bg=bg, rounded=True)
    outs = TH.projected_outcomes(ores[4], cams, ores[5], bg)
    gT = TH.split_flat(T.cpu().numpy(), cams, 1)
    for k in range(len(cams)):
        mx, nfl, mf = TH.check_image(imgs[k].cpu().numpy(), gT[k], ores[0][k], ores[1][k], ores[3][k], outs[k],
                                    what=f"{what} view {k}", max_flag_frac=max_flag_frac)
        note(f"  view {k}: max|d| {mx:.2e}, flagged {nfl} (nearest valid outcome within {mf:.2e})")
    return ores


@pytest.mark.parametrize("case", ["cube10k_256", "mix50k_deg3_480x270"])
def test_end_to_end_matches_oracle(P, torch_cuda, case):
    """Whole pipeline from particle parameters: GPU FP32 footprints vs the FP64 oracle."""
    scenes, cams = _e2e_scenes(case)
    note(f"end-to-end {case}")
    R = P.Rasterizer()
    gsc = [P.GaussianScene.from_host(s) for s in scenes]
    imgs, st = R.render(gsc, cams, bg=(0.0, 0.0, 0.0))
    torch_cuda.cuda.synchronize()
    check_end_to_end(scenes, cams, imgs, st["T"], what=case)


def _grad_scene(deg, n=400, seed=12):
    rng = np.random.default_rng(seed)
    sc = S.uniform_cube_scene(n, seed=seed, log_scale_mean=math.log(0.05), log_scale_std=0.4)
    if deg:
        K = (deg + 1) ** 2
        col = np.zeros((3 * K, n), np.float32)
        col[:3] = sc.color
        col[3:] = rng.normal(0, 0.1, (3 * K - 3, n))
        sc = S.Scene(sc.pos, sc.scale, sc.opacity, col, deg)
    return sc


def unflagged_weights(scenes, cams, rng, bg=(0.0, 0.0, 0.0), max_flag_frac=0.01):
    """Random upstream gradients dL/dC, zero at every pixel the oracle flags end to end
    (where the GPU may take a decision the other way): gradients are then compared with no
    exemption. Returns the per-view weights (FP32) and the oracle's render."""
    ores = O.render_views(scenes, cams, bg=bg, rounded=True)
    Ws = []
    for c, fl in zip(cams, ores[3]):
        assert fl.mean() <= max_flag_frac, float(fl.mean())
        Ws.append((rng.normal(size=(3, c.height, c.width)) * ~fl[None]).astype(np.float32))
    return Ws, ores


def _grads_vs_oracle(g, ref, what=""):
    for name in ("pos", "scale", "opacity", "color"):
        r = TH.grad_check(getattr(g, name).cpu().numpy() if not isinstance(g, dict) else g[name], ref[name],
                         f"{what} {name}")
        note(f"  {name}: max |d| / max|g| {r:.2e}")


@pytest.mark.parametrize("deg", [0, 1, 3])
def test_render_bwd_matches_oracle(P, torch_cuda, deg):
    """Backward pass through the ABI vs the FP64 oracle gradient of L = <W, C>, every
    parameter within 1e-3 |g| + 1e-4 max|g|."""
    torch = torch_cuda
    sc = _grad_scene(deg)
    cams = [S.look_at_camera((0.3, 0.2, 3.0), width=72, height=56),
            S.look_at_camera((-0.4, 0.1, 2.8), width=64, height=64)]
    rng = np.random.default_rng(deg)
    Ws, _ = unflagged_weights([sc, sc], cams, rng)
    note(f"render_bwd deg {deg}")
    R = P.Rasterizer()
    gs = P.GaussianScene.from_host(sc)
    imgs, st = R.render([gs, gs], cams)
    dL = torch.from_numpy(np.concatenate([w.ravel() for w in Ws])).cuda()
    g = R.render_bwd([gs, gs], cams, st["fp"], st["bins"], (0.0, 0.0, 0.0), dL, st["T"], st["n_last"])[0]
    torch.cuda.synchronize()
    ref = O.scene_grads(sc, cams, [w.astype(np.float64) for w in Ws])
    _grads_vs_oracle(g, ref, f"deg {deg}")


def test_autograd_function_and_determinism(P, torch_cuda):
    """The autograd function with an L1 loss: bitwise repeatable, and its gradients equal
    the oracle's L1 gradient. The loss weights out the pixels the oracle flags and those
    whose colour lies within 1e-3 of the target (where the sign of C - target could differ
    between the two sides)."""
    torch = torch_cuda
    sc = _grad_scene(2, n=300, seed=5)
    cams = [S.look_at_camera((0.1, 0.1, 3.0), width=48, height=40) for _ in range(2)]
    cams[1] = S.look_at_camera((-0.3, 0.2, 2.9), width=48, height=40)
    note("autograd + determinism")
    R = P.Rasterizer()
    t = np.random.default_rng(7).uniform(0, 1, (2, 3, 40, 48))
    ores = O.render_views([sc, sc], cams, rounded=True)
    M = np.stack([np.broadcast_to(~ores[3][k][None], (3, 40, 48)) & (np.abs(ores[0][k] - t[k]) > 1e-3)
                  for k in range(2)])
    assert M.mean() > 0.95
    target = torch.from_numpy(t.astype(np.float32)).cuda()
    mask = torch.from_numpy(M.astype(np.float32)).cuda()
    outs = []
    for rep in range(2):
        params = [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
                  for a in (sc.pos, sc.scale, sc.opacity, sc.color)]
        img = P.IsoGSRender.apply(*params, sc.sh_degree, cams, (0.0, 0.0, 0.0), R)
        loss = ((img - target).abs() * mask).sum() / img.numel()
        loss.backward()
        outs.append((img.detach().cpu().numpy(), [p.grad.cpu().numpy() for p in params]))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        np.testing.assert_array_equal(a, b)
    # the L1 gradient through the oracle
    dCs = [M[k] * np.sign(ores[0][k] - t[k]) / t.size for k in range(2)]
    ref = O.scene_grads(sc, cams, dCs)
    _grads_vs_oracle(dict(zip(("pos", "scale", "opacity", "color"), outs[0][1])), ref, "autograd L1")


@pytest.mark.skip(reason="ending the capture of this step (torch.cuda.graph) crashed the process with a segmentation "
                         "fault inside capture_end on the MI355X box; the cause is not found, so the capture of the 3D "
                         "training step is not used (the 2D fit's capture is tested and used)")
def test_training_step_replays_in_a_hip_graph(P, torch_cuda):
    """A forward + backward training step (projection, bin sort, wide forward with
    checkpoints, the library's L1 loss, backward) captured once in a HIP graph with a
    rasterizer that reads no status, replayed several times with eager work and
    synchronisations in between: every replay's image, loss and gradients equal the eager
    step's bitwise (the library's fills are kernels, no memset node is recorded)."""
    torch = torch_cuda
    sc = S.mixture_scene(60_000, seed=12)
    cams = [S.orbit_camera(0.2, 4.0, 320, 240), S.orbit_camera(1.1, 4.0, 320, 240)]
    note("training step in a HIP graph: 60k Gaussians, 2 views of 320x240")
    target = torch.from_numpy(np.random.default_rng(3).uniform(0, 1, (2, 3, 240, 320)).astype(np.float32)).cuda()
    params = [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
              for a in (sc.pos, sc.scale, sc.opacity, sc.color)]
    R = P.Rasterizer()

    def step():
        for q in params:
            q.grad = None
        img = P.IsoGSRender.apply(*params, sc.sh_degree, cams, (0.0, 0.0, 0.0), R)
        loss = P.l1_loss(img, target)
        loss.backward()
        return img, loss

    img, loss = step()                       # eager, checked: sizes the capacity
    ref = (img.detach().clone(), loss.detach().clone(), [q.grad.clone() for q in params])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            step()
    torch.cuda.current_stream().wait_stream(side)
    for q in params:
        q.grad = None
    R.sync_free = True
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_img, g_loss = step()
    g_grads = [q.grad for q in params]       # the graph's own gradient buffers
    R.sync_free = False
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g_img, ref[0]) and torch.equal(g_loss, ref[1]), rep
        for g, r in zip(g_grads, ref[2]):
            assert torch.equal(g, r), rep
        # eager work between replays (another eager step on the same rasterizer)
        e_img, _ = step()
        torch.cuda.synchronize()
        assert torch.equal(e_img.detach(), ref[0])


def test_autograd_output_guarded_against_inplace_changes(P, torch_cuda):
    """The batch returned by the autograd forward is the render buffer itself (no copy),
    which the backward reads; an in-place change of it must make the backward fail
    rather than use the changed image."""
    torch = torch_cuda
    sc = _grad_scene(2, n=300, seed=5)
    cams = [S.look_at_camera((0.1, 0.1, 3.0), width=48, height=40)]
    note("autograd output in-place guard")
    params = [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
              for a in (sc.pos, sc.scale, sc.opacity, sc.color)]
    img = P.IsoGSRender.apply(*params, sc.sh_degree, cams, (0.0, 0.0, 0.0), P.Rasterizer())
    assert img.shape == (1, 3, 40, 48)
    with torch.no_grad():
        img.mul_(2.0)
    with pytest.raises(RuntimeError):
        img.sum().backward()
    with pytest.raises(ValueError):
        P.IsoGSRender.apply(*params, sc.sh_degree, [cams[0], S.look_at_camera((0, 0, 3), width=32, height=40)],
                            (0.0, 0.0, 0.0), P.Rasterizer())


def test_autograd_deferred_capacity_check(P, torch_cuda):
    """The autograd forward does not wait for the capacity status once a capacity is known;
    an overflow is reported by the backward (IsoGSError, capacity grown) and the repeated
    iteration matches a rasterizer that never overflowed."""
    torch = torch_cuda
    sc = _grad_scene(2, n=300, seed=5)
    cams = [S.look_at_camera((0.1, 0.1, 3.0), width=48, height=40)]
    note("autograd deferred capacity check")
    target = torch.rand(1, 3, 40, 48, device="cuda")

    def step(R):
        params = [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
                  for a in (sc.pos, sc.scale, sc.opacity, sc.color)]
        img = P.IsoGSRender.apply(*params, sc.sh_degree, cams, (0.0, 0.0, 0.0), R)
        (img - target).abs().mean().backward()
        return img.detach().cpu().numpy(), [p.grad.cpu().numpy() for p in params]

    good = step(P.Rasterizer())
    R = P.Rasterizer()
    R.capacity = 10                      # known but far too small: the next forward overflows
    with pytest.raises(P.IsoGSError):
        step(R)
    assert R.capacity > 10
    again = step(R)
    np.testing.assert_array_equal(again[0], good[0])
    for a, b in zip(again[1], good[1]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("wide", [False, True], ids=["sequential_fwd", "wide_fwd"])
def test_render_bwd_chunked_long_lists(P, torch_cuda, wide):
    """Tiles with thousands of faint entries: the forward (sequential or wide walk, the
    latter being what training uses) stores checkpoints and the backward walks each long
    list as chunks on separate workgroups; the gradients match the FP64 oracle and the
    single-walk backward (no checkpoints)."""
    torch = torch_cuda
    rng = np.random.default_rng(77)
    base = S.uniform_cube_scene(6000, seed=77, log_scale_mean=math.log(0.06), log_scale_std=0.3)
    opac = rng.uniform(0.005, 0.03, base.pos.shape[1]).astype(np.float32)
    sc = S.Scene(base.pos, base.scale, opac, base.color, 0)
    cams = [S.look_at_camera((0.0, 0.0, 3.2), width=48, height=40)]
    note(f"render_bwd chunked (wide forward: {wide})")
    R = P.Rasterizer()
    gs = P.GaussianScene.from_host(sc)
    imgs, st = R.render([gs], cams, checkpoints=True, wide=wide)
    lens = (st["bins"].ranges[:, 1] - st["bins"].ranges[:, 0]).cpu().numpy()
    assert lens.max() > 3 * 1024, int(lens.max())
    assert int(st["n_last"].max()) > 2048           # pixels keep compositing over many chunks
    Ws, _ = unflagged_weights([sc], cams, rng)
    W = Ws[0]
    dL = torch.from_numpy(W.ravel().copy()).cuda()
    args = ([gs], cams, st["fp"], st["bins"], (0.0, 0.0, 0.0), dL, st["T"], st["n_last"])
    g_chunk = R.render_bwd(*args, image=st["image"], ckpt=st["ckpt"])[0]
    g_whole = R.render_bwd(*args)[0]
    torch.cuda.synchronize()
    ref = O.scene_grads(sc, cams, [W.astype(np.float64)])
    _grads_vs_oracle(g_chunk, ref, "chunked")
    _grads_vs_oracle(g_whole, ref, "whole lists")


def test_render_bwd_checkpoints_all_list_lengths(P, torch_cuda):
    """Lists from a few entries to a few thousand, with and without checkpoints: lists
    shorter than two chunks are walked whole, longer ones as chunks from their
    checkpoints, and both backward passes agree."""
    torch = torch_cuda
    rng = np.random.default_rng(79)
    base = S.uniform_cube_scene(6000, seed=79, log_scale_mean=math.log(0.04), log_scale_std=0.6)
    opac = rng.uniform(0.01, 0.05, base.pos.shape[1]).astype(np.float32)
    sc = S.Scene(base.pos, base.scale, opac, base.color, 0)
    cams = [S.look_at_camera((0.2, -0.1, 3.0), width=96, height=80)]
    note("render_bwd with and without checkpoints, all list lengths")
    R = P.Rasterizer()
    gs = P.GaussianScene.from_host(sc)
    imgs, st = R.render([gs], cams, checkpoints=True)
    lens = (st["bins"].ranges[:, 1] - st["bins"].ranges[:, 0]).cpu().numpy()
    assert ((lens > 256) & (lens < 512)).any() and (lens >= 700).any(), np.sort(lens)[-10:]
    W = rng.normal(size=(3, 80, 96)).astype(np.float32)
    dL = torch.from_numpy(W.ravel().copy()).cuda()
    args = ([gs], cams, st["fp"], st["bins"], (0.0, 0.0, 0.0), dL, st["T"], st["n_last"])
    g_chunk = R.render_bwd(*args, image=st["image"], ckpt=st["ckpt"])[0]
    g_whole = R.render_bwd(*args)[0]
    torch.cuda.synchronize()
    # the same forward decisions on both sides: the walks differ only in how T is
    # recovered (from a checkpoint at most 256 entries back, or by division along the
    # whole list), i.e. by rounding
    for name in ("pos", "scale", "opacity", "color"):
        TH.grad_check(getattr(g_chunk, name).cpu().numpy(), getattr(g_whole, name).cpu().numpy(), name)


def test_wide_forward_independent_of_launch(P, torch_cuda):
    """The wide walk is chosen per tile: a view with tiles of thousands of entries gives
    the same outputs, bitwise, composited alone and as the first of sixteen views in a
    launch of 25,000+ tiles."""
    torch = torch_cuda
    rng = np.random.default_rng(80)
    base = S.uniform_cube_scene(6000, seed=80, log_scale_mean=math.log(0.06), log_scale_std=0.3)
    opac = rng.uniform(0.01, 0.05, base.pos.shape[1]).astype(np.float32)
    sc = S.Scene(base.pos, base.scale, opac, base.color, 0)
    cam0 = S.look_at_camera((0.0, 0.0, 3.2), width=48, height=40)
    cams = [cam0] + [S.orbit_camera(0.3 * i, 4.0, 656, 656) for i in range(15)]
    note("wide forward: alone vs in a 16-view launch")
    R = P.Rasterizer()
    g = P.GaussianScene.from_host(sc)
    outs = []
    for cc in ([cam0], cams):
        fp = R.project([g] * len(cc), cc)
        b = R.bin_sort(fp, [g.n] * len(cc), cc)
        lens = (b.ranges[:, 1] - b.ranges[:, 0]).cpu().numpy()
        assert lens[:9].max() > 3 * 1024
        outs.append(R.render_fwd_ordered(fp, [g.n] * len(cc), b, cc, (0.2, 0.1, 0.3), wide=True))
    torch.cuda.synchronize()
    n0 = 48 * 40
    assert sum(((int(c.width) + 15) // 16) * ((int(c.height) + 15) // 16) for c in cams) > 24576
    assert torch.equal(outs[0][0], outs[1][0][:3 * n0])
    assert torch.equal(outs[0][1], outs[1][1][:n0])
    assert torch.equal(outs[0][2], outs[1][2][:n0])


@pytest.mark.parametrize("wide", [False, True], ids=["pipelined", "wide"])
@pytest.mark.parametrize("scale,opacity", [(0.06, (0.005, 0.03)), (0.25, (0.02, 0.08))])
def test_ordered_forward_long_tiles(P, torch_cuda, scale, opacity, wide):
    """Tiles of thousands of entries: with faint particles no pixel stops, with denser ones
    most pixels stop after their first thousand entries. The longest-first launch equals the
    one-workgroup-per-tile kernel bitwise (pipelined walk) or up to rounding (wide walk:
    per-step products, so a stop decision can move only where T passes within rounding of
    the threshold, a pixel the oracle flags), and both match the oracle."""
    torch = torch_cuda
    rng = np.random.default_rng(78)
    base = S.uniform_cube_scene(6000, seed=78, log_scale_mean=math.log(scale), log_scale_std=0.3)
    opac = rng.uniform(*opacity, base.pos.shape[1]).astype(np.float32)
    sc = S.Scene(base.pos, base.scale, opac, base.color, 0)
    cams = [S.look_at_camera((0.0, 0.0, 3.2), width=48, height=40)]
    note(f"ordered forward, long tiles, opacity {opacity}, wide={wide}")
    R = P.Rasterizer()
    g = P.GaussianScene.from_host(sc)
    fp = R.project([g], cams)
    b = R.bin_sort(fp, [g.n], cams)
    lens = (b.ranges[:, 1] - b.ranges[:, 0]).cpu().numpy()
    assert lens.max() > 3 * 1024
    a = R.render_fwd(fp, [g.n], b, cams, (0.2, 0.1, 0.3))
    c = R.render_fwd_ordered(fp, [g.n], b, cams, (0.2, 0.1, 0.3), wide=wide)
    torch.cuda.synchronize()
    nl_c = c[2].cpu().numpy()
    ores = O.render_views([sc], cams, bg=(0.2, 0.1, 0.3), rounded=True)
    if not wide:
        for x, y in zip(a, c):
            assert torch.equal(x, y)
    else:
        fl = ores[3][0].reshape(-1)
        dimg = np.abs(a[0].cpu().numpy().reshape(3, -1) - c[0].cpu().numpy().reshape(3, -1)).max(axis=0)
        assert dimg[~fl].max() <= 2e-5 and dimg.max() <= 1e-4, (dimg[~fl].max(), dimg.max())
        nl_a = a[2].cpu().numpy()
        assert np.array_equal(nl_a[~fl], nl_c[~fl])
        Ta, Tc = a[1].cpu().numpy(), c[1].cpu().numpy()
        assert np.abs(Ta - Tc)[~fl].max() <= 1e-5
        note(f"  wide vs sequential: max|d| {dimg.max():.2e}, n_last differs at {int((nl_a != nl_c).sum())} px")
    # the denser case stops most pixels after a thousand entries or more, where T carries
    # the most rounding: up to 6% of its pixels are flagged (4.6% measured), each held to
    # one of its valid outcomes
    outs = TH.projected_outcomes(ores[4], cams, ores[5], (0.2, 0.1, 0.3))
    mx, nfl, mf = TH.check_image(c[0].cpu().numpy().reshape(3, 40, 48), c[1].cpu().numpy().reshape(40, 48),
                                ores[0][0], ores[1][0], ores[3][0], outs[0], max_flag_frac=0.06,
                                what=f"long tiles wide={wide}")
    stopped = c[1].cpu().numpy() < 1e-4
    note(f"  max|d| {mx:.2e}, flagged {nfl} (nearest valid outcome within {mf:.2e}), n_last max {int(nl_c.max())}, "
         f"stopped {stopped.mean():.2f}")
    if scale > 0.1:
        assert (nl_c[stopped] > 1024).mean() > 0.5   # most stops come after the first 1024 entries


def _invalid_scene():
    """Valid particles in front of the camera, interleaved with every kind of invalid one:
    non-finite position, scale, opacity or colour; scale <= 0; opacity below 1/255; depth at
    or behind the near plane; footprints with no normal FP32 form (1/s^2 overflowing or
    below the smallest normal)."""
    sc = S.uniform_cube_scene(400, seed=31, log_scale_mean=math.log(0.05), log_scale_std=0.3)
    sc = S.Scene(sc.pos.copy(), sc.scale.copy(), sc.opacity.copy(), sc.color.copy(), 0)
    bad = {}
    kinds = ["pos_nan", "pos_inf", "scale_zero", "scale_neg", "scale_nan", "scale_inf", "opa_low", "opa_nan",
             "color_nan", "color_inf", "behind_near", "behind_camera", "inv_s2_overflow", "inv_s2_denormal"]
    for j, k in enumerate(kinds):
        i = 7 + 13 * j
        bad[k] = i
        if k == "pos_nan":
            sc.pos[0, i] = np.nan
        elif k == "pos_inf":
            sc.pos[1, i] = np.inf
        elif k == "scale_zero":
            sc.scale[i] = 0.0
        elif k == "scale_neg":
            sc.scale[i] = -0.05
        elif k == "scale_nan":
            sc.scale[i] = np.nan
        elif k == "scale_inf":
            sc.scale[i] = np.inf
        elif k == "opa_low":
            sc.opacity[i] = np.float32(1.0 / 256.0)
        elif k == "opa_nan":
            sc.opacity[i] = np.nan
        elif k == "color_nan":
            sc.color[1, i] = np.nan
        elif k == "color_inf":
            sc.color[2, i] = -np.inf
        elif k == "behind_near":
            sc.pos[:, i] = (0.0, 0.0, 3.0 - 0.1)     # depth 0.1 <= near 0.2 for the camera at z = 3
        elif k == "behind_camera":
            sc.pos[:, i] = (0.0, 0.0, 4.0)
        elif k == "inv_s2_overflow":
            sc.scale[i] = np.float32(1e-22)
        elif k == "inv_s2_denormal":
            sc.scale[i] = np.float32(1e19)
    return sc, bad


def test_invalid_particles_culled_like_the_oracle(P, torch_cuda):
    """Per-particle garbage is culled, not an error: each invalid particle gets an all-zero
    record and no tile, exactly where the oracle finds it invisible, and the image of the
    remaining ones matches the oracle end to end."""
    sc, bad = _invalid_scene()
    cam = S.look_at_camera((0.0, 0.0, 3.0), width=96, height=80)
    note(f"invalid particles: {sorted(bad)}")
    R = P.Rasterizer()
    g = P.GaussianScene.from_host(sc)
    fp = R.project([g], [cam])
    torch_cuda.cuda.synchronize()
    rec = fp.record.cpu().numpy()
    tc = fp.tile_count.cpu().numpy()
    pr = O.project64(sc, cam)
    for k, i in bad.items():
        assert not pr.visible[i], k
    assert pr.visible.sum() > 300
    culled = ~pr.visible
    assert (rec[culled] == 0).all() and (tc[culled] == 0).all()
    assert (rec[pr.visible, 3] > 0).all()
    imgs, st = R.render([g], [cam], bg=(0.1, 0.0, 0.2))
    torch_cuda.cuda.synchronize()
    check_end_to_end([sc], [cam], imgs, st["T"], bg=(0.1, 0.0, 0.2), what="invalid particles")
    # and their gradients are exactly zero
    rng = np.random.default_rng(1)
    Ws, _ = unflagged_weights([sc], [cam], rng, bg=(0.1, 0.0, 0.2))
    dL = torch_cuda.from_numpy(Ws[0].ravel().copy()).cuda()
    gr = R.render_bwd([g], [cam], st["fp"], st["bins"], (0.1, 0.0, 0.2), dL, st["T"], st["n_last"])[0]
    torch_cuda.cuda.synchronize()
    for name in ("pos", "scale", "opacity", "color"):
        a = getattr(gr, name).cpu().numpy()
        assert (a[..., culled] == 0).all(), name
    ref = O.scene_grads(sc, [cam], [Ws[0].astype(np.float64)], bg=(0.1, 0.0, 0.2))
    vis = pr.visible
    for name in ("pos", "scale", "opacity", "color"):
        a = getattr(gr, name).cpu().numpy()
        TH.grad_check(a[..., vis], ref[name][..., vis], name)


def test_twenty_views_in_one_call(P, torch_cuda):
    """A call of 20 views (two launch groups of at most 16 views) of two scenes taken in
    turn, at two sizes: forward end to end against the oracle for every view, and the
    backward's per-scene gradients - views of one scene summed across both groups - against
    the oracle's."""
    torch = torch_cuda
    scA = _grad_scene(1, n=500, seed=40)
    scB = _grad_scene(0, n=300, seed=41)
    cams = [S.look_at_camera((0.6 * math.sin(0.31 * i), 0.2 * math.cos(0.7 * i), 3.0 + 0.05 * i),
                             width=56 if i % 3 else 40, height=40 if i % 3 else 48) for i in range(20)]
    scenes = [scA if i % 2 == 0 else scB for i in range(20)]
    note("20 views in one call, two scenes")
    R = P.Rasterizer()
    gA, gB = P.GaussianScene.from_host(scA), P.GaussianScene.from_host(scB)
    gsc = [gA if i % 2 == 0 else gB for i in range(20)]
    imgs, st = R.render(gsc, cams)
    torch.cuda.synchronize()
    check_end_to_end(scenes, cams, imgs, st["T"], what="20 views")
    rng = np.random.default_rng(20)
    Ws = []
    for i in range(20):
        w, _ = unflagged_weights([scenes[i]], [cams[i]], rng)
        Ws.append(w[0])
    dL = torch.from_numpy(np.concatenate([w.ravel() for w in Ws])).cuda()
    grads = R.render_bwd(gsc, cams, st["fp"], st["bins"], (0.0, 0.0, 0.0), dL, st["T"], st["n_last"])
    torch.cuda.synchronize()
    assert len(grads) == 2
    for g, sc, par in ((grads[0], scA, 0), (grads[1], scB, 1)):
        idx = [i for i in range(20) if i % 2 == par]
        ref = O.scene_grads(sc, [cams[i] for i in idx], [Ws[i].astype(np.float64) for i in idx])
        _grads_vs_oracle(g, ref, f"scene {'AB'[par]}")


@pytest.mark.parametrize("family", ["iso", "aniso"])
@pytest.mark.parametrize("walk", ["pipelined", "compact", "wide"])
def test_forward_without_n_last_is_the_same(P, torch_cuda, family, walk):
    """A forward that passes no n_last (no backward follows) composites the same images and
    transmittance bitwise: the walks only skip tracking the last entry. One view takes the
    pipelined walk; twenty 656x656 views are two launch groups, the first sixteen views
    (26896 tiles) in the compact walk, the last four in the pipelined one."""
    torch = torch_cuda
    base = S.uniform_cube_scene(6000, seed=91, log_scale_mean=math.log(0.06), log_scale_std=0.4)
    cams = [S.look_at_camera((0.0, 0.0, 3.2), width=48, height=40)] if walk != "compact" else \
        [S.orbit_camera(0.3 * i, 4.0, 656, 656) for i in range(20)]
    note(f"forward without n_last: {family}, {walk} walk, {len(cams)} view(s)")
    if family == "iso":
        R = P.Rasterizer()
        g = P.GaussianScene.from_host(base)
    else:
        R = P.AnisoRasterizer()
        g = P.AnisoGaussianScene.from_host(S.aniso_from_iso(base))
    fp = R.project([g] * len(cams), cams)
    b = R.bin_sort(fp, [g.n] * len(cams), cams)
    full = R.render_fwd_ordered(fp, [g.n] * len(cams), b, cams, (0.2, 0.1, 0.3), wide=walk == "wide")
    bare = R.render_fwd_ordered(fp, [g.n] * len(cams), b, cams, (0.2, 0.1, 0.3), wide=walk == "wide", last=False)
    torch.cuda.synchronize()
    assert bare[2] is None
    assert int((full[2] > 0).sum()) > 0
    assert torch.equal(full[0], bare[0])
    assert torch.equal(full[1], bare[1])
    if family == "iso":
        # the one-workgroup-per-tile kernel without n_last as well
        spat = R.render_fwd(fp, [g.n] * len(cams), b, cams, (0.2, 0.1, 0.3), last=False)
        torch.cuda.synchronize()
        assert spat[2] is None
        if walk != "wide":
            assert torch.equal(spat[0], full[0]) and torch.equal(spat[1], full[1])
