"""GPU checks of the serving path: the longest-list-first compositing launch equals
the one-workgroup-per-tile launch bitwise, and every request served in a mixed,
continuously batched stream gets exactly the image it gets when rendered alone."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import scenegen as S

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible device"
    import paper_2403_14244_amd as P
    return P


def _scenes():
    return {"small": S.mixture_scene(20_000, seed=21, log_scale_mean=math.log(0.01)),
            "mid": S.mixture_scene(60_000, seed=22),
            "cube": S.uniform_cube_scene(8000, seed=23, log_scale_mean=math.log(0.03))}


@pytest.mark.parametrize("views", ["three_small", "sixteen_640"])
def test_ordered_equals_per_tile_launch(P, views):
    """Longest-list-first dispatch against the spatial one-workgroup-per-tile launch, bitwise:
    three small views (pipelined walk) and sixteen 640x640 views (25600 tiles, above the
    pipelined walk's limit: compact walk)."""
    import torch
    note(f"ordered == per-tile ({views})")
    if views == "three_small":
        sc = S.mixture_scene(100_000, seed=3)
        sizes = [(640, 360), (512, 512), (333, 190)]
    else:
        sc = S.mixture_scene(60_000, seed=4)
        sizes = [(640, 640)] * 16
    cams = [S.orbit_camera(0.4 * i, 4.0, w, h) for i, (w, h) in enumerate(sizes)]
    R = P.Rasterizer()
    g = P.GaussianScene.from_host(sc)
    fp = R.project([g] * len(cams), cams)
    b = R.bin_sort(fp, [g.n] * len(cams), cams)
    a = R.render_fwd(fp, [g.n] * len(cams), b, cams, (0.1, 0.2, 0.3))
    c = R.render_fwd_ordered(fp, [g.n] * len(cams), b, cams, (0.1, 0.2, 0.3))
    torch.cuda.synchronize()
    for x, y in zip(a, c):
        assert torch.equal(x, y)


@pytest.mark.parametrize("walk", ["pipelined", "compact", "wide"])
def test_workgroup_stamps(P, walk):
    """ISOGS_FWD_TIMES: the images are unchanged, every workgroup that composited a non-empty
    list leaves start < end, the others {0, 0}; the compact and pipelined walks take one
    workgroup per tile, so exactly the non-empty tiles are stamped (twenty views: two
    launch groups, the second group's stamps from pair 5 t on)."""
    import torch
    note(f"workgroup stamps ({walk})")
    sc = S.mixture_scene(60_000, seed=7)
    sizes = {"pipelined": [(640, 360)] * 2, "compact": [(640, 640)] * 20, "wide": [(640, 360)] * 2}[walk]
    cams = [S.orbit_camera(0.3 * i, 4.0, w, h) for i, (w, h) in enumerate(sizes)]
    R = P.Rasterizer()
    g = P.GaussianScene.from_host(sc)
    fp = R.project([g] * len(cams), cams)
    b = R.bin_sort(fp, [g.n] * len(cams), cams)
    wide = walk == "wide"
    a = [x.clone() for x in R.render_fwd_ordered(fp, [g.n] * len(cams), b, cams, wide=wide)]
    img, T, nl, st = R.render_fwd_ordered(fp, [g.n] * len(cams), b, cams, wide=wide, times=True)
    torch.cuda.synchronize()
    for x, y in zip(a, (img, T, nl)):
        assert torch.equal(x, y)
    st = st.cpu().numpy()
    lens = (b.ranges[:, 1] - b.ranges[:, 0]).cpu().numpy()
    stamped = st[:, 0] != 0
    assert np.all(st[stamped, 1] > st[stamped, 0]) and np.all(st[~stamped] == 0)
    if walk == "wide":
        assert stamped.sum() >= (lens > 0).sum()
    else:
        # group g's workgroups at pairs 5 t0 + b; one per tile
        tiles = [((w + 15) // 16) * ((h + 15) // 16) for w, h in sizes]
        t0 = 0
        for v0 in range(0, len(sizes), 16):
            n = sum(tiles[v0:v0 + 16])
            grp = stamped[5 * t0:5 * t0 + n]
            assert grp.sum() == (lens[t0:t0 + n] > 0).sum()
            assert not stamped[5 * t0 + n:5 * (t0 + n)].any()
            t0 += n
    span = (st[stamped, 1].max() - st[stamped, 0].min()) * 10e-3
    note(f"  {int(stamped.sum())} workgroups, mean {(st[stamped, 1] - st[stamped, 0]).mean() * 10e-3:.1f} us, "
         f"launch span {span:.1f} us")


def test_served_images_equal_alone_and_in_mix(P):
    import torch
    from paper_2403_14244_amd.serving import GpuExecutor, Request, Server
    note("serving: alone vs mixed")
    host = _scenes()
    dev = {k: P.GaussianScene.from_host(v) for k, v in host.items()}
    rng = np.random.default_rng(5)
    res = [(96, 64), (128, 128), (200, 120)]
    reqs, t = [], 0.0
    for i in range(40):
        t += rng.exponential(1 / 2000.0)
        w, h = res[int(rng.integers(3))]
        reqs.append(Request(rid=i, scene=list(host)[int(rng.integers(3))],
                            cam=S.orbit_camera(float(rng.uniform(0, 2 * math.pi)), 4.0, w, h), arrival=t))
    ex = GpuExecutor(dev)
    ex.calibrate(reqs)
    srv = Server(ex, pool_bytes=1 << 30, max_batch=8, max_inflight=2, keep_results=True)
    st = srv.run(reqs)
    torch.cuda.synchronize()
    note(f"  served {st['requests']} in {st['batches']} batches, mean {st['mean_batch']:.2f}")
    assert st["requests"] == 40 and st["mean_batch"] > 1.0
    R = P.Rasterizer()
    for r in reqs:
        alone, _ = R.render([dev[r.scene]], [r.cam], wide=True)   # the serving walk
        assert torch.equal(alone[0], r.result), r.rid
    # and a few against the oracle (end to end, FP64; near a decision, one of the valid
    # results)
    from tests import _helpers as TH
    for r in reqs[:3]:
        ores = O.render_views([host[r.scene]], [r.cam], rounded=True)
        outs = TH.projected_outcomes(ores[4], [r.cam], ores[5])
        img = r.result.cpu().numpy()
        ok_px = ~ores[3][0]
        d = np.abs(img.astype(np.float64) - ores[0][0]).max(axis=0)
        assert d[ok_px].max() <= 1e-4, (r.rid, float(d[ok_px].max()))
        assert ores[3][0].mean() <= 0.01
        for y, x in zip(*np.nonzero(ores[3][0])):
            cands, ok = outs[0](int(y), int(x))
            assert ok and min(float(np.abs(img[:, y, x] - c).max()) for c, _, _ in cands) <= 1e-4, (r.rid, y, x)


def test_batches_overlap_on_the_device(P):
    """Continuous batching with two slots: a burst of requests fills both slots, and the
    device spans of batches on the two streams intersect (their work overlaps on the
    device), while every served image stays bitwise equal to the image rendered alone."""
    import torch
    from paper_2403_14244_amd.serving import GpuExecutor, Request, Server
    note("serving: device overlap of in-flight batches")
    # batches of six 1080p views of 1M-particle scenes: milliseconds of device work each,
    # well above the host's time to queue the next batch
    host = {"a": S.mixture_scene(1_000_000, seed=24), "b": S.mixture_scene(1_000_000, seed=25)}
    dev = {k: P.GaussianScene.from_host(v) for k, v in host.items()}
    rng = np.random.default_rng(6)
    def trace(first):
        return [Request(rid=first + i, scene="ab"[i % 2],
                        cam=S.orbit_camera(float(rng.uniform(0, 2 * math.pi)), 4.0, 1920, 1080), arrival=0.0)
                for i in range(36)]
    warm, reqs = trace(0), trace(100)
    ex = GpuExecutor(dev, record_spans=True)
    ex.calibrate(warm + reqs)
    # a first pass with the same batches sizes both slots' workspaces and leaves the kept
    # images' blocks in the allocator's cache of each stream, so that queueing a batch is
    # host work only (a fresh device allocation would stall the host between batches)
    Server(ex, pool_bytes=1 << 32, max_batch=6, max_inflight=2, keep_results=True).run(warm)
    torch.cuda.synchronize()
    for r in warm:
        r.result = None
    ex.spans.clear()
    srv = Server(ex, pool_bytes=1 << 32, max_batch=6, max_inflight=2, keep_results=True)
    st = srv.run(reqs)
    ov = ex.device_overlap()
    note(f"  {st['batches']} batches, overlap {ov}, host submits (ms) "
         f"{[round(r.submit * 1e3, 2) for r in reqs[::6]]}")
    assert st["batches"] >= 4 and ov["batches"] == st["batches"]
    assert ov["overlapping_pairs"] >= 1 and ov["overlap_ms"] > 0.0
    R = P.Rasterizer()
    for r in reqs[::5]:
        alone, _ = R.render([dev[r.scene]], [r.cam], wide=True)
        assert torch.equal(alone[0], r.result), r.rid
