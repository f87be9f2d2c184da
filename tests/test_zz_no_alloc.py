"""isogs_bin_sort_static (the bin sort whose scratch is the library's static per-GPU array)
against isogs_bin_sort with a caller workspace, through the C ABI: bit-exact keys, particle
indices, tile ranges, offsets, count and status, on two calls in a row, the second with a
smaller input (the array keeps the first call's contents)."""
import ctypes
import math
import sys

import numpy as np
import pytest

import scenegen as S

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _bins_host(b):
    import torch
    torch.cuda.synchronize()
    n = int(b.count.item())
    cap = b.capacity
    m = min(n, cap)
    return dict(count=n, status=int(b.status.item()), keys=b.keys[:m].cpu().numpy().copy(),
                pidx=b.pidx[:m].cpu().numpy().copy(), ranges=b.ranges.cpu().numpy().copy(),
                offsets=b.offsets.cpu().numpy().copy())


def _both(P, R, scenes, cams, capacity):
    """The same footprints binned by both entry points into separate output bins."""
    from paper_2403_14244_amd import _abi as A
    from paper_2403_14244_amd.rasterizer import _alloc_bins, _p, _stream, tiles_of
    import torch
    gs = [P.GaussianScene.from_host(s) for s in scenes]
    fp = R.project(gs, cams)
    npv = [g.n for g in gs]
    n_total, tiles = sum(npv), sum(tiles_of(c) for c in cams)
    ref = _alloc_bins(capacity, n_total, tiles, R.device, with_keys=True)
    stat = _alloc_bins(capacity, n_total, tiles, R.device, with_keys=True)
    # make stale outputs visible: the static call must write everything it reports
    for t in (stat.pidx, stat.keys, stat.ranges, stat.offsets):
        t.fill_(-7)
    L = A.lib()
    carr, npa = A.camera_array(cams), A.int_array(npv)
    need = ctypes.c_size_t(0)
    A.check(L.isogs_bin_sort(ctypes.byref(fp.abi()), npa, carr, len(cams), ctypes.byref(ref.abi()), None,
                             ctypes.byref(need), _stream()))
    assert need.value <= A.ISOGS_STATIC_SCRATCH_BYTES, need.value
    ws = torch.empty(need.value, dtype=torch.uint8, device=R.device)
    have = ctypes.c_size_t(ws.numel())
    A.check(L.isogs_bin_sort(ctypes.byref(fp.abi()), npa, carr, len(cams), ctypes.byref(ref.abi()), _p(ws),
                             ctypes.byref(have), _stream()))
    A.check(L.isogs_bin_sort_static(ctypes.byref(fp.abi()), npa, carr, len(cams), ctypes.byref(stat.abi()),
                                    _stream()))
    return _bins_host(ref), _bins_host(stat), need.value


def _same(a, b, what):
    assert a["count"] == b["count"] and a["status"] == b["status"] == 0, (what, a["count"], b["count"], a["status"],
                                                                          b["status"])
    for k in ("keys", "pidx", "ranges", "offsets"):
        assert np.array_equal(a[k], b[k]), (what, k)


def test_static_bin_sort_matches_the_workspace_call_twice():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible device"
    import paper_2403_14244_amd as P
    R = P.Rasterizer()
    # first call: three 1280x720 views of a 200k mixture scene (several sort tiles, long lists)
    big = S.mixture_scene(200_000, seed=3)
    cams1 = [S.orbit_camera(2 * math.pi * i / 3, 4.0, 1280, 720) for i in range(3)]
    note("static bin sort: 200k x 3 views 1280x720")
    a, b, need1 = _both(P, R, [big] * 3, cams1, capacity=1_500_000)
    _same(a, b, "first call")
    assert a["count"] > 100_000
    note(f"  {a['count']} entries, scratch {need1} bytes: bit-exact")
    # second call, smaller: one ragged view of a 3000-particle scene; the array still holds
    # the first call's data, which must not leak into this result
    small = S.uniform_cube_scene(3000, seed=1, log_scale_mean=math.log(0.03))
    cams2 = [S.look_at_camera((0.0, 0.0, 3.0), width=100, height=70)]
    note("static bin sort: 3000 x 1 view 100x70")
    a2, b2, need2 = _both(P, R, [small], cams2, capacity=40_000)
    assert need2 < need1
    _same(a2, b2, "second call")
    note(f"  {a2['count']} entries, scratch {need2} bytes: bit-exact")


def test_static_bin_sort_reports_capacity_overflow_like_the_workspace_call():
    import torch
    import paper_2403_14244_amd as P
    R = P.Rasterizer()
    small = S.uniform_cube_scene(3000, seed=1, log_scale_mean=math.log(0.03))
    cams = [S.look_at_camera((0.0, 0.0, 3.0), width=100, height=70)]
    note("static bin sort: overflowing capacity")
    from paper_2403_14244_amd import _abi as A
    gs = P.GaussianScene.from_host(small)
    fp = R.project([gs], cams)
    ref = R.bin_sort(fp, [gs.n], cams, check=False, capacity=100)
    st = R.bin_sort_static(fp, [gs.n], cams, capacity=100)
    torch.cuda.synchronize()
    assert int(ref.status.item()) == int(st.status.item()) == A.ISOGS_ERR_CAPACITY
    assert int(ref.count.item()) == int(st.count.item()) > 100


def test_static_bin_sort_rejects_sizes_beyond_the_array():
    import paper_2403_14244_amd as P
    from paper_2403_14244_amd import _abi as A
    R = P.Rasterizer()
    small = S.uniform_cube_scene(100, seed=1)
    cams = [S.look_at_camera((0.0, 0.0, 3.0), width=64, height=64)]
    gs = P.GaussianScene.from_host(small)
    fp = R.project([gs], cams)
    with pytest.raises(A.IsoGSError) as e:
        R.bin_sort_static(fp, [gs.n], cams, capacity=8_000_000)
    assert e.value.code == A.ISOGS_ERR_WORKSPACE
