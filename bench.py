"""Benchmark of the isotropic-splatting rasterizer on one MI355X.

Workload (the forward metric): 1,000,000 isotropic Gaussians (64 clusters + 8 sphere
shells, degree-3 SH colour) rendered from 100 orbit views at 1920x1080. One step renders
all 100 views: projection, binning, radix sort and compositing for every view, inputs
resident in HBM. `value` is forward megapixels per second over the timed steps.

Also reported: fwd+bwd iterations/s (one 1080p view of the same scene through the
autograd function with an L1 loss), per-stage times, the roofline of the dominant
kernel (measured with HIP events on the launch stream) and the FP64 CPU oracle timed on
a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# room for the forward's four streams in HIP's per-process pool of hardware queues (4 by
# default, shared with torch's own streams; streams that share a queue run in turn); the
# serving slots' streams get queues outside the pool; set before the HIP runtime starts
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

HBM_PEAK_GBS = 8000.0
# published FP32 vector peak (packed FMA), and without packed instructions (this build emits
# none): 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3
VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--views", type=int, default=100)
    ap.add_argument("--batch-views", type=int, default=10)
    ap.add_argument("--streams", type=int, default=4,
                    help="HIP streams the forward batches alternate over (sort of one batch overlaps "
                         "compositing of another)")
    ap.add_argument("--gaussians", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--train-iters", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="length of the request trace of the serving measurement (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-inflight", type=int, default=2,
                    help="batches in flight at once (one HIP stream each)")
    ap.add_argument("--serve-warmup", type=int, default=1000, help="warm-up requests before the measured trace")
    ap.add_argument("--serve-sweep", default="1000,3000,10000",
                    help="extra arrival rates (req/s), 500 requests each, for the batch size and latency at load")
    ap.add_argument("--only-serving", action="store_true", help="run only the serving measurement")
    ap.add_argument("--only-stress", action="store_true",
                    help="run only the 6M 4K stress workload and print its JSON object")
    ap.add_argument("--only-field2d", action="store_true",
                    help="run only the 2D fit (2000 kernels, 512x512) and print its JSON object")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="skip the 500k 4x720p training step and the 6M 4K stress fwd+bwd")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for counter runs: one copy kernel of known size, then one forward call")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the solo per-stage measurement (the phase the roofline figures come from), "
                         "for a kernel trace of exactly those launches")
    return ap.parse_args()


COPY_BYTES = 512 << 20
FLOPS_PER_PAIR = 9   # dx, dy, dx^2 + dy^2 (3), times -log2(e)/s^2, exp, times o, clamp
# reverse walk, per (pixel, entry) pair: alpha as above (9), T before the entry (2), its weight
# (1), dC/dalpha per channel and its dot with dL/dC (14), light from behind (6), colour
# gradient (3), kernel and opacity gradients (9)
BWD_FLOPS_PER_PAIR = 44


def composite_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "raster.h", "composite.hip"):
        h.update(open(os.path.join(ROOT, "paper_2403_14244_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(bytes_per_launch_alg):
    """HBM bytes per compositing launch from the committed counter summary, if it was taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_composite_fwd_mix1m_1080p.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("sources_digest") != composite_sources_digest():
        return None
    return d["hbm_bytes_per_launch"]


def walk_pairs(T, n_last, ranges, cams, tile_base0=0):
    """Evaluated (pixel, entry) pairs of the plain tiled walk: every pixel walks its tile's
    list until it terminates (then up to its last contributor) or to the end."""
    import torch
    total = 0
    pix_off, tile_off = 0, tile_base0
    for c in cams:
        W, H = int(c.width), int(c.height)
        TX, TY = (W + 15) // 16, (H + 15) // 16
        lens = (ranges[tile_off:tile_off + TX * TY, 1] - ranges[tile_off:tile_off + TX * TY, 0]).long()
        ys = torch.arange(H, device=T.device) // 16
        xs = torch.arange(W, device=T.device) // 16
        tid = (ys[:, None] * TX + xs[None, :]).reshape(-1)
        t = T[pix_off:pix_off + W * H]
        nl = n_last[pix_off:pix_off + W * H].long()
        walk = torch.where(t < 1e-4, nl, lens[tid])
        total += int(walk.sum().item())
        pix_off += W * H
        tile_off += TX * TY
    return total


def bwd_pairs(n_last):
    """(pixel, entry) pairs of the reverse walk: every pixel walks back from its last
    contributing entry."""
    return int(n_last.long().sum().item())


def hold_stream():
    """Queue a spin kernel on the current stream (5M cycles of the device clock: about 2 ms
    at 2.4 GHz) so that the host enqueues the launches that follow while the device is busy:
    HIP events placed after it then time the device's work alone, with no host launch
    latency between a synchronisation and the first kernel."""
    import torch
    torch.cuda._sleep(5_000_000)


def solo_stages(R, gs, batches, dL_seed=7):
    """Every stage of the benchmark call alone on one stream, with HIP events on that
    stream around each library call: projection, bin sort, longest-first compositing (as
    the benchmark calls it, without checkpoints) and the backward pass (random dL/dimage,
    from an untimed forward with checkpoints, as training runs it), per batch of views.
    Returns the mean time per call of each stage (ms), and the work of the compositing
    walks."""
    import torch
    st = {k: [] for k in ("project", "bin_sort", "render_fwd", "render_bwd")}
    fwd_pairs = bwd_p = entries = 0
    gen = torch.Generator(device=gs.pos.device)
    gen.manual_seed(dL_seed)
    for bc in batches:
        npv = [gs.n] * len(bc)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        hold_stream()
        ev[0].record()
        fp = R.project([gs] * len(bc), bc)
        ev[1].record()
        bins = R.bin_sort(fp, npv, bc, check=False)
        ev[2].record()
        # the forward as the benchmark launches it (no checkpoints, no n_last); then, untimed, the
        # training forward with checkpoints that the backward starts its chunks from
        img, T, n_last = R.render_fwd_ordered(fp, npv, bins, bc, last=False)
        ev[3].record()
        ck = R.checkpoint_buffer(bins)
        img, T, n_last = R.render_fwd_ordered(fp, npv, bins, bc, ckpt=ck)
        dL = torch.randn(img.shape, device=img.device, generator=gen)
        e_b0, e_b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e_b0.record()
        R.render_bwd([gs] * len(bc), bc, fp, bins, (0.0, 0.0, 0.0), dL, T, n_last, image=img, ckpt=ck)
        e_b1.record()
        torch.cuda.synchronize()
        bins.verify()
        st["project"].append(ev[0].elapsed_time(ev[1]))
        st["bin_sort"].append(ev[1].elapsed_time(ev[2]))
        st["render_fwd"].append(ev[2].elapsed_time(ev[3]))
        st["render_bwd"].append(e_b0.elapsed_time(e_b1))
        fwd_pairs += walk_pairs(T, n_last, bins.ranges, bc)
        bwd_p += bwd_pairs(n_last)
        entries += bins.n_entries()
        del ck, dL, img, T, n_last, bins, fp
    nb = len(batches)
    return ({k: float(np.mean(v)) for k, v in st.items()}, fwd_pairs / nb, bwd_p / nb, entries / nb)


def size_capacity(R, gs, batches):
    """Entry capacity of the rasterizer sized with a checked bin sort of every batch (it only
    grows), so that the unchecked timed calls fit."""
    for bc in batches:
        R.bin_sort(R.project([gs] * len(bc), bc), [gs.n] * len(bc), bc, check=True)


def stage_rooflines(ms, fwd_pairs, bwd_pairs_, entries, n, views, pixels, tiles, sh_degree):
    """Per-stage figures of one call from its solo time: algorithmic work (bytes or flops per
    unit as stated in the design notes), achieved rate and its fraction of the published
    peaks (HBM 8 TB/s; FP32 157.3 TFLOP/s, 78.6 without packed instructions)."""
    K = (sh_degree + 1) ** 2
    out = {}
    proj_b = n * (20 + 12 * K) + n * views * 40
    sort_b = entries * 24
    fwd_b = entries * 36 + pixels * 16 + tiles * 8   # the benchmark launch writes no n_last
    for name, alg_b in (("project", proj_b), ("bin_sort", sort_b)):
        gbs = alg_b / (ms[name] * 1e-3) / 1e9
        out[name] = {"us": round(ms[name] * 1e3, 1), "bound": "hbm", "alg_bytes": int(alg_b),
                     "alg_gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    for name, pairs, fpp, alg_b in (("render_fwd", fwd_pairs, FLOPS_PER_PAIR, fwd_b),
                                    ("render_bwd", bwd_pairs_, BWD_FLOPS_PER_PAIR, None)):
        tf = pairs * fpp / (ms[name] * 1e-3) / 1e12
        out[name] = {"us": round(ms[name] * 1e3, 1), "bound": "alu", "pairs": int(pairs), "flops_per_pair": fpp,
                     "tflops": round(tf, 3), "frac_fp32_peak": round(tf / FP32_PEAK_TFLOPS, 4),
                     "frac_nonpacked": round(tf / VALU_PEAK_TFLOPS, 4)}
        if alg_b:
            out[name]["alg_bytes"] = int(alg_b)
            out[name]["alg_gbs"] = round(alg_b / (ms[name] * 1e-3) / 1e9, 1)
    return out


def poisson_trace(n, rate_hz, scene_names, resolutions, seed=4, radius=4.0, start_id=0):
    """Serving requests: exponential inter-arrival times (mean 1/rate), a uniformly chosen
    resident scene, an orbit camera at a uniform angle and a uniformly chosen resolution."""
    import scenegen as S
    from paper_2403_14244_amd.serving import Request
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        name = scene_names[int(rng.integers(len(scene_names)))]
        th = float(rng.uniform(0, 2 * math.pi))
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        out.append(Request(rid=start_id + i, scene=name, cam=S.orbit_camera(th, radius, w, h), arrival=t))
    return out


def serving_benchmark(args, dev):
    """Four resident scenes (200k, 1M, 2M, 3M Gaussians), Poisson arrivals, mixed
    resolutions, continuous batching on two streams; latency = completion - arrival."""
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    from paper_2403_14244_amd.serving import GpuExecutor, Server
    sizes = {"mix200k": (200_000, 10), "mix1m": (1_000_000, 11), "mix2m": (2_000_000, 12), "mix3m": (3_000_000, 13)}
    scenes = {k: P.GaussianScene.from_host(S.mixture_scene(n, seed=sd), dev) for k, (n, sd) in sizes.items()}
    res = [(512, 512), (1280, 720), (1920, 1080)]
    n = max(1, int(args.serve_seconds * args.serve_rate))
    warm = poisson_trace(args.serve_warmup, args.serve_rate, list(scenes), res, seed=3)
    reqs = poisson_trace(n, args.serve_rate, list(scenes), res, seed=4, start_id=1_000_000)
    rates = [float(x) for x in args.serve_sweep.split(",") if x.strip()]
    sweeps = {r: poisson_trace(500, r, list(scenes), res, seed=5 + k, start_id=2_000_000 + 1000 * k)
              for k, r in enumerate(rates)}
    ex = GpuExecutor(scenes, dev, n_streams=args.serve_inflight, record_spans=True)
    ex.calibrate(warm + reqs + [q for v in sweeps.values() for q in v])
    log(f"serving: {len(warm)} warm-up requests ...")
    Server(ex, pool_bytes=16 << 30, max_batch=16, max_inflight=args.serve_inflight).run(warm)
    torch.cuda.synchronize()
    ex.spans.clear()
    log(f"serving: trace of {len(reqs)} requests at {args.serve_rate:g}/s ...")
    srv = Server(ex, pool_bytes=16 << 30, max_batch=16, max_inflight=args.serve_inflight)
    st = srv.run(reqs)
    ov = ex.device_overlap()
    sel = [r.latency * 1e3 for r in reqs if r.scene == "mix1m" and r.cam.width == 1920]
    st["p99_ms_1080p_1m"] = float(np.percentile(sel, 99)) if sel else None
    st["rate_hz"] = args.serve_rate
    st["warmup_requests"] = len(warm)
    st["scenes"] = {k: v[0] for k, v in sizes.items()}
    st["capacity_overflows"] = ex.overflows
    st["device_overlap"] = {"overlapping_batch_pairs": ov["overlapping_pairs"],
                            "ms_two_batches_on_device": round(ov["overlap_ms"], 2),
                            "ms_device_busy": round(ov["busy_ms"], 2)}
    st.pop("pool_bytes", None)
    sweep_out = {}
    for r, trace in sweeps.items():
        ex.spans.clear()
        s2 = Server(ex, pool_bytes=16 << 30, max_batch=16, max_inflight=args.serve_inflight).run(trace)
        o2 = ex.device_overlap()
        sweep_out[f"{int(r)}_req_per_s"] = {"requests": s2["requests"], "mean_batch": round(s2["mean_batch"], 3),
                                            "p50_ms": round(s2["p50_ms"], 3), "p99_ms": round(s2["p99_ms"], 3),
                                            "mpix_per_s": round(s2["mpix_per_s"], 1),
                                            "overlapping_batch_pairs": o2["overlapping_pairs"],
                                            "ms_two_batches_on_device": round(o2["overlap_ms"], 2),
                                            "ms_device_busy": round(o2["busy_ms"], 2)}
    st["rate_sweep"] = sweep_out
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}


def cube_workload(dev, iters=200):
    """The small forward workload: 10,000 particles uniform in the cube, one 256x256 view from
    distance 3 (RGB). Forward Mpix/s over `iters` renders, and each stage's solo time."""
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    scene = S.workload_scene("cube10k_256")
    cams = S.workload_cameras("cube10k_256")
    gs = P.GaussianScene.from_host(scene, dev)
    R = P.Rasterizer(dev, headroom=1.1)
    for _ in range(5):
        R.render([gs], cams, check=False)
    R.render([gs], cams, check=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        R.render([gs], cams, check=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    solo_stages(R, gs, [cams])
    ms, fwd_pairs, bwd_p, entries = solo_stages(R, gs, [cams] * 20)
    return {"workload": "cube10k_256", "gaussians": 10_000, "width": 256, "height": 256,
            "fwd_mpix_per_s": round(256 * 256 / dt / 1e6, 1), "fwd_us_per_render": round(dt * 1e6, 1),
            "entries": int(entries), "walk_pairs": int(fwd_pairs),
            "stage_us_solo": {k: round(v * 1e3, 1) for k, v in ms.items()}}


def training_workload(dev, iters=20):
    """The training step as the workload states it: 500k Gaussians, targets rendered from the
    ground truth at views 0, 25, 50, 75 of the orbit at 1280x720, parameters from a jittered
    copy, L1 loss through the autograd function; iterations per second."""
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    gt = S.mixture_scene(500_000, seed=0)
    init = S.jitter_scene(gt, seed=1)
    cams = S.workload_cameras("mix500k_720p_x4")
    R = P.Rasterizer(dev, headroom=1.1)
    targets = torch.stack(R.render([P.GaussianScene.from_host(gt, dev)] * len(cams), cams)[0])
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).requires_grad_(True)
              for a in (init.pos, init.scale, init.opacity, init.color)]

    def step():
        for q in params:
            q.grad = None
        img = P.IsoGSRender.apply(*params, init.sh_degree, cams, (0.0, 0.0, 0.0), R)
        loss = P.l1_loss(img, targets)
        loss.backward()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    return {"workload": "mix500k_720p_x4", "iters_per_s": round(1.0 / dt, 2), "ms_per_iter": round(dt * 1e3, 3),
            "views": len(cams), "width": 1280, "height": 720, "gaussians": 500_000}


def stress_workload(dev, iters=3):
    """6M Gaussians (70% in 16 tight clusters), SH3, 8 views at 3840x2160: forward and
    backward against L1 targets of the ground truth, parameters from a jittered copy; ms per
    iteration, and the tile list lengths that skew the load."""
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    gt = S.stress_scene(6_000_000, seed=5)
    init = S.jitter_scene(gt, seed=1)
    cams = S.workload_cameras("stress6m_4k_x8")
    R = P.Rasterizer(dev, headroom=1.1)
    imgs, st = R.render([P.GaussianScene.from_host(gt, dev)] * len(cams), cams)
    targets = torch.stack(imgs)
    lens = (st["bins"].ranges[:, 1] - st["bins"].ranges[:, 0]).long()
    nz = lens[lens > 0].float()
    hist = torch.bincount(torch.floor(torch.log2(nz)).long(), minlength=18).tolist()
    lists = {"tiles": int(lens.numel()), "occupied": int(nz.numel()), "entries": int(lens.sum()),
             "mean": round(float(nz.mean()), 1), "p50": int(nz.median()), "p99": int(torch.quantile(nz, 0.99)),
             "max": int(nz.max()), "log2_histogram": {f"[{1 << i},{2 << i})": c for i, c in enumerate(hist) if c}}
    del imgs, st
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).requires_grad_(True)
              for a in (init.pos, init.scale, init.opacity, init.color)]

    def step():
        for q in params:
            q.grad = None
        img = P.IsoGSRender.apply(*params, init.sh_degree, cams, (0.0, 0.0, 0.0), R)
        loss = P.l1_loss(img, targets)
        loss.backward()

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    # the forward alone (projection, bin sort, compositing) of the same 8 views
    g_init = P.GaussianScene(*(q.detach() for q in params), init.sh_degree)
    fwd = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        hold_stream()
        e0.record()
        R.render([g_init] * len(cams), cams, check=False)
        e1.record()
        torch.cuda.synchronize()
        fwd.append(e0.elapsed_time(e1))
    # load balance of the compositing launch: per-workgroup clock stamps (100 MHz) of the
    # forward's compact walk and of the training step's wide walk, over the workgroups that
    # composited a non-empty list
    fp = R.project([g_init] * len(cams), cams)
    bins = R.bin_sort(fp, [g_init.n] * len(cams), cams)
    balance = {}
    for name, wide in (("compact_walk", False), ("wide_walk", True)):
        st = R.render_fwd_ordered(fp, [g_init.n] * len(cams), bins, cams, wide=wide, times=True)[3]
        st = st.cpu().numpy()
        on = st[:, 0] != 0
        dur = (st[on, 1] - st[on, 0]) * 1e-2     # us
        balance[name] = {"workgroups": int(on.sum()), "mean_us": round(float(dur.mean()), 2),
                         "p99_us": round(float(np.percentile(dur, 99)), 1), "max_us": round(float(dur.max()), 1),
                         "max_over_mean": round(float(dur.max() / dur.mean()), 1),
                         "launch_span_us": round(float((st[on, 1].max() - st[on, 0].min()) * 1e-2), 1)}
    del fp, bins
    return {"workload": "stress6m_4k_x8", "fwd_bwd_ms_per_iter": round(dt * 1e3, 2),
            "fwd_ms": round(sorted(fwd)[1], 2), "views": len(cams), "width": 3840, "height": 2160,
            "gaussians": 6_000_000, "mpix_per_s_fwd": round(len(cams) * 3840 * 2160 / (sorted(fwd)[1] * 1e-3) / 1e6, 1),
            "tile_lists": lists, "composite_workgroup_time": balance}


def aniso_workload(dev, scene_iso, cams, batch_views=10, fwd_views=20, train_iters=10):
    """The paper's comparison of isotropic and anisotropic kernels (Table 1, Table 2, the
    "about 100X" of the abstract and Section 3) on this library's own kernels, both
    families built from the same walks: the isotropic scene of the benchmark, the same
    particles as anisotropic ones (identity rotation, sigma on every axis: each particle's
    full sigma^2 J J^T footprint) and an anisotropic scene of the same layout with random
    orientations and per-axis scales. Per variant: forward Mpix/s over `fwd_views` orbit
    views at 1080p in calls of `batch_views` (one stream), entries per view, and fwd+bwd
    iterations/s at one 1080p view with the L1 loss through the autograd function."""
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    n = scene_iso.n
    variants = {"iso": scene_iso, "aniso_same_particles": S.aniso_from_iso(scene_iso),
                "aniso_random": S.aniso_mixture_scene(n, seed=0)}
    views = cams[:fwd_views]
    batches = [views[i:i + batch_views] for i in range(0, len(views), batch_views)]
    W, H = int(views[0].width), int(views[0].height)
    target = torch.rand(1, 3, H, W, device=dev)
    out = {}
    for name, sc in variants.items():
        an = name != "iso"
        R = (P.AnisoRasterizer if an else P.Rasterizer)(dev, headroom=1.1)
        g = (P.AnisoGaussianScene if an else P.GaussianScene).from_host(sc, dev)

        def fwd(check):
            ents = []
            for bc in batches:
                fp = R.project([g] * len(bc), bc)
                bins = R.bin_sort(fp, [g.n] * len(bc), bc, check=check)
                R.render_fwd_ordered(fp, [g.n] * len(bc), bins, bc, last=False)
                ents.append(bins)
            return ents

        fwd(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            bins_all = fwd(False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        for b in bins_all:
            b.verify()
        entries = sum(b.n_entries() for b in bins_all) / len(views)
        params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).requires_grad_(True)
                  for a in ((sc.pos, sc.rot, sc.scale, sc.opacity, sc.color) if an else
                            (sc.pos, sc.scale, sc.opacity, sc.color))]
        fn = P.AnisoGSRender if an else P.IsoGSRender
        Rt = (P.AnisoRasterizer if an else P.Rasterizer)(dev, headroom=1.1)

        def step():
            for q in params:
                q.grad = None
            img = fn.apply(*params, sc.sh_degree, views[:1], (0.0, 0.0, 0.0), Rt)
            P.l1_loss(img, target).backward()

        for _ in range(2):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(train_iters):
            step()
        torch.cuda.synchronize()
        it = train_iters / (time.perf_counter() - t0)
        out[name] = {"fwd_mpix_per_s": round(len(views) * W * H / dt / 1e6, 1),
                     "fwd_ms_per_view": round(dt * 1e3 / len(views), 3), "entries_per_view": round(entries),
                     "fwd_bwd_iters_per_s": round(it, 1)}
        del R, Rt, params, g, bins_all
        torch.cuda.empty_cache()
    iso = out["iso"]
    for k in ("aniso_same_particles", "aniso_random"):
        out[k]["iso_speedup_fwd"] = round(iso["fwd_mpix_per_s"] / out[k]["fwd_mpix_per_s"], 3)
        out[k]["iso_speedup_fwd_bwd"] = round(iso["fwd_bwd_iters_per_s"] / out[k]["fwd_bwd_iters_per_s"], 3)
    out["workload"] = f"mix1m_1080p: {len(views)} orbit views, calls of {batch_views}; fwd+bwd at 1 view, L1"
    return out


def field2d_workload(dev, iters=100):
    """The paper's 2D experiment on a synthetic stand-in: fit 2000 weighted isotropic kernels
    (random initialisation) to a procedural 512x512 RGB image with the paper's loss,
    0.8 L1 + 0.2 (1 - SSIM), and Adam, at support radii D = 15 and 50 px. One iteration:
    binning, kernel sum, loss, gradients, optimizer step. Also the kernel sum's and its
    backward's times alone (HIP events on their stream), and the same number of
    iterations from the quadtree initialisation (at most 2000 leaves) instead of the
    random one, and the rate of the step captured once in a HIP graph and replayed."""
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    tgt_np = S.field2d_target(512, 512)
    mu0, s0, a0 = S.field2d_init(tgt_np, 2000)
    tgt = torch.from_numpy(tgt_np).to(dev)
    res = {"workload": "field2d_fit512_k2000", "width": 512, "height": 512, "particles": 2000}
    # the paper's tree initialisation of the same budget, timed on the device
    P.tree_init(tgt, 2000, 64, 2, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = P.tree_init(tgt, 2000, 64, 2, 1e-3)
    res["tree_init_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    res["tree_init_particles"] = int(tree[1].shape[0])

    def fit(R, start, n):
        mu, s, a = (x.clone().requires_grad_(True) for x in start)
        opt = torch.optim.Adam([mu, s, a], lr=0.02)
        first = None
        for _ in range(n):
            opt.zero_grad(set_to_none=True)
            loss = P.l1_ssim_loss(P.Field2DRender.apply(mu, s, a, R), tgt)
            loss.backward()
            opt.step()
            with torch.no_grad():
                s.clamp_(min=0.3)
            first = float(loss.detach()) if first is None else first
        return first, float(loss.detach())

    for D in (15.0, 50.0):
        tree_first, tree_after = fit(P.Field2DRenderer(512, 512, D, device=dev), tree, iters + 6)
        R = P.Field2DRenderer(512, 512, D, device=dev)
        mu, s, a = (torch.from_numpy(x.copy()).to(dev).requires_grad_(True) for x in (mu0, s0, a0))
        opt = torch.optim.Adam([mu, s, a], lr=0.02)

        def step():
            opt.zero_grad(set_to_none=True)
            img = P.Field2DRender.apply(mu, s, a, R)
            loss = P.l1_ssim_loss(img, tgt)
            loss.backward()
            opt.step()
            with torch.no_grad():
                s.clamp_(min=0.3)
            return loss

        l0 = float(step().detach())
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            loss = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / iters
        with torch.no_grad():
            fp, bins = R.bin(mu.detach(), s.detach(), a.detach())
            w = torch.sign(R.render(fp, bins, 2000) - tgt) / tgt.numel()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            hold_stream()
            ev[0].record()
            for _ in range(20):
                R.render(fp, bins, 2000)
            ev[1].record()
            for _ in range(20):
                R.grads(fp, bins, 2000, w)
            ev[2].record()
            torch.cuda.synchronize()
        entries = bins.n_entries()
        fwd_us = ev[0].elapsed_time(ev[1]) * 1e3 / 20
        # the same step captured once in a HIP graph and replayed (no host work per step)
        gparams = [torch.from_numpy(x.copy()).to(dev).requires_grad_(True) for x in (mu0, s0, a0)]
        gopt = torch.optim.Adam(gparams, lr=0.02, capturable=True)
        Rg = P.Field2DRenderer(512, 512, D, device=dev)

        def gstep():
            gopt.zero_grad(set_to_none=True)
            gl = P.l1_ssim_loss(P.Field2DRender.apply(*gparams, Rg), tgt)
            gl.backward()
            gopt.step()
            with torch.no_grad():
                gparams[1].clamp_(min=0.3)
            return gl

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                gstep()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gloss = gstep()
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            graph.replay()
        torch.cuda.synchronize()
        gdt = (time.perf_counter() - t0) / iters
        # Table 2's comparison: the same fit with anisotropic kernels (angle 0, both scales
        # sigma at the start; angle and scales optimised), same loss, optimizer and support
        Ra = P.Field2DAnisoRenderer(512, 512, D, device=dev)
        amu, aa = (torch.from_numpy(x.copy()).to(dev).requires_grad_(True) for x in (mu0, a0))
        ath = torch.zeros(2000, device=dev, requires_grad=True)
        asc = torch.from_numpy(np.stack([s0, s0])).to(dev).requires_grad_(True)
        aopt = torch.optim.Adam([amu, ath, asc, aa], lr=0.02)

        def astep():
            aopt.zero_grad(set_to_none=True)
            al = P.l1_ssim_loss(P.Field2DAnisoRender.apply(amu, ath, asc, aa, Ra), tgt)
            al.backward()
            aopt.step()
            with torch.no_grad():
                asc.clamp_(min=0.3)
            return al

        for _ in range(6):
            astep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            aloss = astep()
        torch.cuda.synchronize()
        adt = (time.perf_counter() - t0) / iters
        with torch.no_grad():
            afp, acc, abins = Ra.bin(amu.detach(), ath.detach(), asc.detach(), aa.detach())
            aw = torch.sign(Ra.render(afp, acc, abins, 2000) - tgt) / tgt.numel()
            aev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            hold_stream()
            aev[0].record()
            for _ in range(20):
                Ra.render(afp, acc, abins, 2000)
            aev[1].record()
            for _ in range(20):
                Ra.grads(amu.detach(), ath.detach(), asc.detach(), aa.detach(), afp, acc, abins, aw)
            aev[2].record()
            torch.cuda.synchronize()
        aniso = {"iters_per_s": round(1.0 / adt, 1), "ms_per_iter": round(adt * 1e3, 3),
                 "loss_after": round(float(aloss.detach()), 5), "entries": abins.n_entries(),
                 "fwd_kernel_us": round(aev[0].elapsed_time(aev[1]) * 1e3 / 20, 2),
                 "bwd_kernels_us": round(aev[1].elapsed_time(aev[2]) * 1e3 / 20, 2),
                 "iso_speedup": round(adt / dt, 3)}
        res[f"d{int(D)}"] = {"iters_per_s": round(1.0 / dt, 1), "ms_per_iter": round(dt * 1e3, 3),
                             "s_per_2000_iters": round(2000 * dt, 2), "loss": "0.8 L1 + 0.2 (1 - SSIM)",
                             "loss_first": round(l0, 5), "loss_after": round(float(loss.detach()), 5), "entries": entries,
                             "fwd_kernel_us": round(fwd_us, 2),
                             "bwd_kernels_us": round(ev[1].elapsed_time(ev[2]) * 1e3 / 20, 2),
                             "fwd_pairs_per_s": round(entries * 256 / (fwd_us * 1e-6), 1),
                             "graph_iters_per_s": round(1.0 / gdt, 1),
                             "graph_loss_after": round(float(gloss.detach()), 5),
                             "tree_init_loss_first": round(tree_first, 5),
                             "tree_init_loss_after": round(tree_after, 5), "aniso": aniso}
    return res


_CPU = {}


def _cpu_workers():
    """Host cores this process may use, at most 16 (the CPU share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _cpu_tiles(args):
    """Worker: composites its tiles with the FP64 oracle until the deadline."""
    import oracle as O
    tiles, deadline = args
    pr, bins, cam = _CPU["pr"], _CPU["bins"], _CPU["cam"]
    done, pix = 0, 0
    for k in tiles:
        if time.perf_counter() > deadline:
            break
        TXc = (cam.width + 15) // 16
        tx, ty = int(k) % TXc, int(k) // TXc
        O.render64_tiled(pr.u, pr.v, pr.s, pr.opacity, pr.rgb, bins, 0, cam.width, cam.height, tiles=[(tx, ty)])
        done += 1
        pix += len(O.tile_pixels(tx, ty, cam.width, cam.height)[0])
    return done, pix


def _cpu_rows(args):
    """Worker: the untiled oracle (every pixel over every visible particle) on some rows."""
    import oracle as O
    key, rows = args
    pr, cam = _CPU[key]
    O.render64_untiled(pr, cam.width, cam.height, rows=rows)
    return len(rows) * cam.width


def cpu_baseline(scene, cam, budget_s):
    """The FP64 oracle on the host's cores (a pool of worker processes, one BLAS thread
    each): one view of the benchmark workload - full projection and binning of all
    particles, then the tiled compositing of seeded-random tiles until the time budget is
    spent, extrapolated to the full frame; also the untiled definition (every pixel over
    every visible particle) on the 10k-particle 256x256 workload's full frame and on a 64x64
    centre crop of the benchmark view, and one iteration of the 2D fit."""
    import multiprocessing as mp
    import oracle as O
    import scenegen as S
    from threadpoolctl import threadpool_limits
    workers = _cpu_workers()
    ctx = mp.get_context("fork")
    out = {}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pr = O.project64(scene, cam)
        t1 = time.perf_counter()
        bins = O.bin_sort_ref(O.f32_views([pr], [cam]))
        t2 = time.perf_counter()
        TX, TY = O.tile_grid(cam.width, cam.height)
        order = np.random.default_rng(0).permutation(TX * TY)
        _CPU.update(pr=pr, bins=bins, cam=cam)
        # untiled legs: the 10k-particle 256x256 frame and a 64x64 crop of this view
        c1_scene, c1_cam = S.workload_scene("cube10k_256"), S.workload_cameras("cube10k_256")[0]
        _CPU["cube"] = (O.project64(c1_scene, c1_cam), c1_cam)
        crop = cam.shifted(cam.width // 2 - 32, cam.height // 2 - 32, 64, 64)
        _CPU["crop"] = (O.project64(scene, crop), crop)
        with ctx.Pool(workers) as pool:
            deadline = time.perf_counter() + budget_s
            ts = time.perf_counter()
            res = pool.map(_cpu_tiles, [(order[w::workers], deadline) for w in range(workers)])
            t_render = time.perf_counter() - ts
            done_tiles, pix = sum(r[0] for r in res), sum(r[1] for r in res)
            legs = {}
            for key in ("cube", "crop"):
                H = _CPU[key][1].height
                ts = time.perf_counter()
                npx = sum(pool.map(_cpu_rows, [(key, np.arange(w, H, workers)) for w in range(workers)]))
                legs[key] = (npx, time.perf_counter() - ts)
        # the 2D fit: one iteration (kernel sum, loss gradient, parameter gradients) per radius
        from oracle import field2d64 as F2
        from oracle import ssim64 as Q2
        tgt = S.field2d_target(512, 512)
        mu, sg, amp = S.field2d_init(tgt, 2000)
        f2 = {}
        for D in (15.0, 50.0):
            ts = time.perf_counter()
            _, w = Q2.l1_ssim_loss64(F2.render_field64(mu, sg, amp, 512, 512, D), tgt)
            F2.field_grads64(mu, sg, amp, 512, 512, D, w)
            f2[f"d{int(D)}_s_per_iter"] = round(time.perf_counter() - ts, 3)
    total_pix = cam.width * cam.height
    per_view = (t1 - t0) + (t2 - t1) + t_render * (total_pix / max(pix, 1))
    out = dict(value=total_pix / per_view / 1e6, unit="Mpix/s", cores=workers, kind="oracle",
               sample=f"1 view of 1920x1080 / 1M Gaussians: FP64 projection and binning of all particles "
                      f"({t1 - t0:.1f}s + {t2 - t1:.1f}s, one process), tiled compositing of {done_tiles} random "
                      f"tiles ({pix} px) in {t_render:.1f}s on {workers} worker processes, extrapolated to the "
                      f"full frame",
               os_cpu_count=os.cpu_count(),
               untiled_cube10k_256_full_frame={"mpix_per_s": round(legs["cube"][0] / legs["cube"][1] / 1e6, 5),
                                               "s": round(legs["cube"][1], 2), "pixels": legs["cube"][0],
                                               "pairs": int(_CPU["cube"][0].visible.sum()) * legs["cube"][0]},
               untiled_mix1m_1080p_crop64={"mpix_per_s": round(legs["crop"][0] / legs["crop"][1] / 1e6, 6),
                                           "s": round(legs["crop"][1], 2), "pixels": legs["crop"][0]},
               field2d_fit512_k2000=f2)
    _CPU.clear()
    return out


def roofline_phase(R, gs, batches, args):
    """Solo stage times and the roofline of the dominant kernel (compositing)."""
    size_capacity(R, gs, batches)
    solo_stages(R, gs, batches[:1])       # warm: workspaces sized, code loaded
    ms, fwd_pairs, bwd_p, entries = solo_stages(R, gs, batches)
    B = len(batches[0])
    pixels = B * args.width * args.height
    tiles = B * ((args.width + 15) // 16) * ((args.height + 15) // 16)
    stages = stage_rooflines(ms, fwd_pairs, bwd_p, entries, gs.n, B, pixels, tiles, gs.sh_degree)
    fwd = stages["render_fwd"]
    comp_bytes = entries * 36 + pixels * 16 + tiles * 8   # image, T (no n_last)
    achieved = fwd_pairs * FLOPS_PER_PAIR / (ms["render_fwd"] * 1e-3) / 1e12
    roof = dict(kernel="composite_fwd_ordered_kernel<false>", bound="alu", achieved=achieved, peak=FP32_PEAK_TFLOPS,
                unit="TFLOP/s", frac=achieved / FP32_PEAK_TFLOPS, traffic=measured_traffic(comp_bytes),
                frac_nonpacked=achieved / VALU_PEAK_TFLOPS, nonpacked_peak=round(VALU_PEAK_TFLOPS, 2),
                launch_ms=ms["render_fwd"], launches=len(batches), measured="solo launches, HIP events on the "
                "launch stream (isogs_render_fwd_ordered as the benchmark calls it: the tile queue's three small "
                "kernels and the compositing kernel)", pairs_per_launch=fwd_pairs, flops_per_pair=FLOPS_PER_PAIR, alg_bytes_per_launch=comp_bytes,
                hbm_gbs_alg=comp_bytes / (ms["render_fwd"] * 1e-3) / 1e9, views_per_launch=B)
    log(f"solo stages per {B}-view call: " + ", ".join(f"{k} {v['us']} us" for k, v in stages.items()))
    log(f"composite: {ms['render_fwd'] * 1e3:.0f} us/launch alone, {fwd_pairs:.3e} pairs, {achieved:.2f} TFLOP/s "
        f"({roof['frac']:.3f} of {FP32_PEAK_TFLOPS}, {roof['frac_nonpacked']:.3f} of {VALU_PEAK_TFLOPS:.1f})")
    return roof, stages


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (rendering and "
              "serving would shard by view and request, training by views with one gradient all-reduce)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import scenegen as S
    import paper_2403_14244_amd as P
    if args.only_field2d:
        print(json.dumps(field2d_workload("cuda")), flush=True)
        return
    if args.only_stress:
        torch.cuda.set_device(0)
        print(json.dumps(stress_workload(torch.device("cuda:0"))), flush=True)
        return
    if args.only_serving:
        torch.cuda.set_device(0)
        print(json.dumps({"serving": serving_benchmark(args, torch.device("cuda:0"))}), flush=True)
        return

    t = time.perf_counter()
    scene = S.mixture_scene(args.gaussians, seed=0)
    cams = [S.orbit_camera(2.0 * math.pi * i / args.views, 4.0, args.width, args.height) for i in range(args.views)]
    log(f"scene generated in {time.perf_counter() - t:.1f}s")
    cpu = None
    if not args.no_cpu_baseline and not args.pmc_probe and not args.roofline_only:
        # before the GPU is touched: the oracle's worker processes fork from this one
        log(f"cpu baseline ({_cpu_workers()} worker processes) ...")
        cpu = cpu_baseline(scene, cams[0], args.cpu_seconds)
        cpu["value"] = round(cpu["value"], 5)
        log(f"cpu baseline: {cpu}")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    gs = P.GaussianScene.from_host(scene, dev)
    R = P.Rasterizer(dev, headroom=1.1)
    B = args.batch_views
    batches = [cams[i:i + B] for i in range(0, len(cams), B)]
    # batch k runs on stream k mod S with its own rasterizer (workspace), so that the
    # memory-bound sort of one batch overlaps the ALU-bound compositing of another
    main = torch.cuda.current_stream()
    streams = [main] + [torch.cuda.Stream(device=dev) for _ in range(max(args.streams, 1) - 1)]
    rasters = [R] + [P.Rasterizer(dev, headroom=1.1) for _ in streams[1:]]

    # size the entry capacity on the warm-up pass
    def forward_step(check, spans=True):
        stage = dict(project=[], bin_sort=[], render_fwd=[])
        bins_all = []
        go = torch.cuda.Event()
        go.record(main)
        for s in streams[1:]:
            s.wait_event(go)
        for k, bc in enumerate(batches):
            s, Rk = streams[k % len(streams)], rasters[k % len(streams)]
            with torch.cuda.stream(s):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if spans else [None] * 4
                mark = (lambda e: e.record(s)) if spans else (lambda e: None)
                scenes = [gs] * len(bc)
                mark(ev[0])
                fp = Rk.project(scenes, bc)
                mark(ev[1])
                bins = Rk.bin_sort(fp, [gs.n] * len(bc), bc, check=check)
                mark(ev[2])
                Rk.render_fwd_ordered(fp, [gs.n] * len(bc), bins, bc, last=False)
                mark(ev[3])
            if spans:
                stage["project"].append((ev[0], ev[1]))
                stage["bin_sort"].append((ev[1], ev[2]))
                stage["render_fwd"].append((ev[2], ev[3]))
            bins_all.append(bins)
        for s in streams[1:]:
            done = torch.cuda.Event()
            done.record(s)
            main.wait_event(done)
        return stage, bins_all

    if args.pmc_probe:
        size_capacity(R, gs, batches[:1])
        solo_stages(R, gs, batches[:1])       # sizes the workspaces
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                      # plain copy: COPY_BYTES read + COPY_BYTES written
        torch.cuda.synchronize()
        # one call of every stage, as the roofline phase makes it (fwd with checkpoints, bwd)
        ms, fwd_pairs, bwd_p, entries = solo_stages(R, gs, batches[:1])
        print(json.dumps({"pmc_probe": True, "copy_bytes": COPY_BYTES, "views": len(batches[0]),
                          "entries": entries, "sources_digest": composite_sources_digest()}))
        return

    if args.roofline_only:
        roof, stages_solo = roofline_phase(R, gs, batches, args)
        print(json.dumps({"roofline": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in roof.items()},
                          "stages_solo_per_call": stages_solo}), flush=True)
        return

    for _ in range(max(args.warmup, 1)):
        _, bins_all = forward_step(check=True)
    torch.cuda.synchronize()
    entries = [b.n_entries() for b in bins_all]
    log(f"warm-up done: entries per batch {entries}, capacity {[r.capacity for r in rasters]}, "
        f"{len(streams)} stream(s)")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, bins_all = forward_step(check=False, spans=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for b in bins_all:
        b.verify()
    ms_step = elapsed / args.steps * 1e3
    mpix = args.steps * args.views * args.width * args.height / elapsed / 1e6
    # the stage spans of one more step, with timing events between the stages (outside the
    # timed region: the events are instrumentation, not part of the workload)
    st, _ = forward_step(check=False, spans=True)
    torch.cuda.synchronize()
    stage_ms = {k: sum(a.elapsed_time(b) for a, b in st[k]) for k in st}
    log(f"forward: {ms_step:.2f} ms/step, {mpix:.1f} Mpix/s, stages of one instrumented step {stage_ms}")

    # per-stage rooflines from solo launches (nothing else on the GPU), one call per batch;
    # the dominant kernel is compositing, bound by the FP32 VALU: work = evaluated (pixel,
    # entry) pairs of the plain tiled walk x 9 flops
    roof, stages_solo = roofline_phase(R, gs, batches, args)

    # fwd+bwd iterations per second: one 1080p view, L1 loss, autograd
    cam1 = [cams[0]]
    target = torch.rand(1, 3, args.height, args.width, device=dev)
    params = [gs.pos.clone().requires_grad_(True), gs.scale.clone().requires_grad_(True),
              gs.opacity.clone().requires_grad_(True), gs.color.clone().requires_grad_(True)]
    Rt = P.Rasterizer(dev, headroom=1.1)

    def train_iter():
        for q in params:
            q.grad = None   # what an optimizer's zero_grad() does before each step
        img = P.IsoGSRender.apply(*params, gs.sh_degree, cam1, (0.0, 0.0, 0.0), Rt)
        loss = P.l1_loss(img, target)
        loss.backward()
        return loss

    def train_rate():
        for _ in range(2):
            train_iter()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.train_iters):
            train_iter()
        torch.cuda.synchronize()
        return args.train_iters / (time.perf_counter() - t1)

    # compositing of a single view is tail-bound by its longest tiles: the longest-first
    # launch is measured beside the spatial one-workgroup-per-tile launch
    it_by_kernel = {}
    for ordered in (False, True):
        Rt.ordered_fwd = ordered
        it_by_kernel["ordered" if ordered else "per_tile"] = round(train_rate(), 2)
    it_s = it_by_kernel["ordered"]   # the rasterizer's default for render()
    log(f"fwd+bwd: {it_s:.1f} it/s ({it_by_kernel})")

    extra = {}
    if not args.no_extra_workloads:
        del Rt, params
        torch.cuda.empty_cache()
        log("cube10k_256 forward ...")
        extra["cube10k_256"] = cube_workload(dev)
        log(f"cube10k_256: {extra['cube10k_256']}")
        log("training workload (500k, 4 x 1280x720) ...")
        extra["training_500k_720p_x4"] = training_workload(dev)
        log(f"training workload: {extra['training_500k_720p_x4']}")
        torch.cuda.empty_cache()
        log("stress workload (6M, 8 x 3840x2160) ...")
        extra["stress_6m_4k_x8"] = stress_workload(dev)
        log(f"stress workload: {extra['stress_6m_4k_x8']}")
        torch.cuda.empty_cache()
        log("iso vs aniso (1M, 1080p) ...")
        extra["iso_vs_aniso"] = aniso_workload(dev, scene, cams)
        log(f"iso vs aniso: {extra['iso_vs_aniso']}")
        torch.cuda.empty_cache()
        log("2D fit (2000 kernels, 512x512) ...")
        extra["field2d_fit512_k2000"] = field2d_workload(dev)
        log(f"2D fit: {extra['field2d_fit512_k2000']}")

    serving = None
    if args.serve_seconds > 0:
        log("serving ...")
        serving = serving_benchmark(args, dev)
        log(f"serving: p50 {serving['p50_ms']} ms, p99 {serving['p99_ms']} ms, "
            f"1080p/1M p99 {serving['p99_ms_1080p_1m']} ms, {serving['mpix_per_s']} Mpix/s")

    out = {
        "metric": "forward Mpix/s at 1920x1080, 1M Gaussians (SH3), 100 orbit views",
        "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded generator; no dataset)",
        "config": {"workload": "mix1m_1080p_x100", "gaussians": args.gaussians, "views": args.views,
                   "width": args.width, "height": args.height, "sh_degree": 3, "views_per_call": B,
                   "streams": len(streams)},
        "stage_ms_per_step": {k: round(v, 3) for k, v in stage_ms.items()},
        "entries_per_view": round(float(np.mean(entries)) / B),
        "fwd_bwd_iters_per_s": round(it_s, 2),
        "fwd_bwd_iters_per_s_by_fwd_kernel": it_by_kernel,
        "roofline": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in roof.items()},
        "stages_solo_per_call": stages_solo,
        "stage_span_us_per_view_overlapped": {k: round(v * 1e3 / args.views, 1) for k, v in stage_ms.items()},
        "serving": serving,
        **extra,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
