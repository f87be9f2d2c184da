"""Serving loop: resident scenes, memory-admitted continuous batching, latency statistics.

Requests (scene, camera, arrival time) are admitted in arrival order into batches of
views. A batch is formed whenever an execution slot is free, from every request that has
arrived and fits the memory pool; requests that arrive while batches are running are
admitted as soon as a slot and pool memory free up, and up to `max_inflight` batches run
concurrently on separate HIP streams, so their work overlaps on the device. Each batch is
one projection (grouped by scene), one bin sort and one longest-list-first compositing launch
(tiles of at least 2048 entries with the wide walk, a decision of each tile alone, so a
request's image does not depend on the batch it ran in).

The scheduler is written against a small executor interface so that its admission,
batching and statistics logic also runs on the CPU with a simulated executor and a
virtual clock (see `SimulatedExecutor`); `GpuExecutor` drives the C ABI.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass

import numpy as np


@dataclass
class Request:
    rid: int
    scene: str
    cam: object
    arrival: float                 # seconds on the server clock
    submit: float | None = None
    done: float | None = None
    batch: int | None = None
    result: object = None

    @property
    def pixels(self) -> int:
        return int(self.cam.width) * int(self.cam.height)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.002))


class VirtualClock:
    """Deterministic clock for tests: sleeping advances time."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float):
        self.t = max(self.t, t)


class Executor:
    """What the scheduler needs from a device."""

    def bytes_needed(self, req: Request) -> int:
        raise NotImplementedError

    def submit(self, batch: list[Request]):
        """Starts a batch asynchronously; returns a handle."""
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> None:
        """Called once poll() is true: stores each request's result."""
        raise NotImplementedError

    def next_event_time(self, handle) -> float | None:
        """For simulated executors: when the batch completes (None if unknown)."""
        return None


class Server:
    def __init__(self, executor: Executor, pool_bytes: int, max_batch: int = 16, max_inflight: int = 2,
                 clock=None, keep_results: bool = False):
        self.ex = executor
        self.pool = int(pool_bytes)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.clock = clock or RealClock()
        self.keep_results = keep_results
        self.used = 0
        self.peak_used = 0
        self.batches = []          # (size, submit time, bytes)

    def run(self, requests: list[Request]) -> dict:
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        ready: deque[Request] = deque()
        inflight = []              # (handle, batch, bytes)
        finished = []
        nb = 0
        for r in pending:
            if self.ex.bytes_needed(r) > self.pool:
                raise ValueError(f"request {r.rid} needs more memory than the whole pool")
        while pending or ready or inflight:
            now = self.clock.now()
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            # admit: one new batch per free slot, FIFO, bounded by the pool
            while ready and len(inflight) < self.max_inflight:
                batch, need = [], 0
                while ready and len(batch) < self.max_batch:
                    b = self.ex.bytes_needed(ready[0])
                    if self.used + need + b > self.pool:
                        break
                    need += b
                    batch.append(ready.popleft())
                if not batch:
                    break
                t = self.clock.now()
                for r in batch:
                    r.submit, r.batch = t, nb
                h = self.ex.submit(batch)
                self.used += need
                self.peak_used = max(self.peak_used, self.used)
                inflight.append((h, batch, need))
                self.batches.append((len(batch), t, need))
                nb += 1
            # completions
            still = []
            for h, batch, need in inflight:
                if self.ex.poll(h):
                    self.ex.finish(h)
                    t = self.clock.now()
                    for r in batch:
                        r.done = t
                        if not self.keep_results:
                            r.result = None
                    finished.extend(batch)
                    self.used -= need
                else:
                    still.append((h, batch, need))
            progressed = len(still) != len(inflight)
            inflight = still
            if not progressed:
                # nothing completed: wait for the next arrival or completion
                wake = [pending[0].arrival] if pending else []
                for h, _, _ in inflight:
                    te = self.ex.next_event_time(h)
                    if te is not None:
                        wake.append(te)
                nxt = min(wake) if wake else self.clock.now() + 1e-4
                if inflight and not any(self.ex.next_event_time(h) is not None for h, _, _ in inflight):
                    nxt = min(nxt, self.clock.now() + 5e-5)
                self.clock.sleep_until(nxt)
        return self.stats(finished)

    def stats(self, finished: list[Request]) -> dict:
        if not finished:
            return dict(requests=0)
        lat = np.array([r.latency for r in finished]) * 1e3
        first = min(r.arrival for r in finished)
        last = max(r.done for r in finished)
        pix = sum(r.pixels for r in finished)
        sizes = [b[0] for b in self.batches]
        by_res = {}
        for r in finished:
            by_res.setdefault(f"{r.cam.width}x{r.cam.height}", []).append(r.latency * 1e3)
        return dict(requests=len(finished), p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), max_ms=float(lat.max()),
                    mpix_per_s=pix / (last - first) / 1e6, wall_s=last - first,
                    batches=len(sizes), mean_batch=float(np.mean(sizes)), peak_pool_bytes=self.peak_used,
                    pool_bytes=self.pool,
                    p99_ms_by_resolution={k: float(np.percentile(v, 99)) for k, v in sorted(by_res.items())})


class SimulatedExecutor(Executor):
    """CPU stand-in: a batch takes base + per_mpix * megapixels seconds on the clock.
    Optionally renders each request with a supplied function (e.g. the oracle)."""

    def __init__(self, clock, scenes_n: dict, base=1e-3, per_mpix=2e-4, render=None):
        self.clock = clock
        self.scenes_n = scenes_n
        self.base = base
        self.per_mpix = per_mpix
        self.render = render
        self.n_submitted = 0

    def bytes_needed(self, req):
        return 40 * self.scenes_n[req.scene] + 20 * req.pixels

    def submit(self, batch):
        self.n_submitted += 1
        t = self.clock.now()
        return dict(batch=batch, t_done=t + self.base + self.per_mpix * sum(r.pixels for r in batch) / 1e6)

    def poll(self, h):
        return self.clock.now() >= h["t_done"]

    def next_event_time(self, h):
        return h["t_done"]

    def finish(self, h):
        if self.render is not None:
            for r in h["batch"]:
                r.result = self.render(r)


def _own_streams(n, device):
    """`n` HIP streams created for this executor by the library (default priority, each on a
    hardware queue of its own), wrapped as torch streams. Streams from the process's shared
    pool of queues (torch's own, plain hipStreamCreate) can share a queue, which runs their
    work in turn."""
    import ctypes
    import torch
    from . import _abi as A
    handles, streams = [], []
    with torch.cuda.device(device):
        for _ in range(n):
            h = ctypes.c_void_p()
            A.check(A.lib().isogs_stream_create(ctypes.byref(h)))
            handles.append(h.value)
            streams.append(torch.cuda.ExternalStream(h.value, device=device))
    return handles, streams


class GpuExecutor(Executor):
    """Runs batches through the C ABI on `n_streams` HIP streams (default priority).

    Batches of different slots overlap on the device only where their streams sit on
    different hardware queues: the slots' streams come from `isogs_stream_create`, which
    gives each a queue of its own outside the pool of GPU_MAX_HW_QUEUES queues that HIP
    shares among the process's other streams."""

    def __init__(self, scenes: dict, device="cuda", n_streams=2, headroom=1.3, record_spans=False):
        import torch
        from .rasterizer import Rasterizer
        self.torch = torch
        # with record_spans, each batch's device span (events before its first and after
        # its last launch, on its stream) is kept for device_overlap()
        self.record_spans = record_spans
        self.spans = []
        self.scenes = scenes                    # name -> GaussianScene (resident)
        self.device = torch.device(device)
        # the streams live as long as the process: events that torch records on them (its
        # pinned-memory allocator's, for the status copies) may be queried after the
        # executor is gone, and a destroyed stream would leave them dangling
        self._handles, self.streams = _own_streams(n_streams, self.device)
        self.busy = [False] * n_streams
        self.rasters = [Rasterizer(self.device) for _ in range(n_streams)]
        # one pinned {count, status} word pair per slot, reused: a slot runs one batch at a time
        self.status_host = [torch.empty(2, dtype=torch.int32, pin_memory=True) for _ in range(n_streams)]
        self.headroom = headroom
        self.entries_per_view = {}              # (scene, W, H) -> entries seen
        self.overflows = 0

    def _key(self, r):
        return (r.scene, int(r.cam.width), int(r.cam.height))

    def calibrate(self, requests):
        """Measures entries per (scene, resolution) once, synchronously."""
        seen = {}
        for r in requests:
            seen.setdefault(self._key(r), r)
        for k, r in seen.items():
            R = self.rasters[0]
            g = self.scenes[r.scene]
            fp = R.project([g], [r.cam])
            b = R.bin_sort(fp, [g.n], [r.cam])
            self.entries_per_view[k] = b.n_entries()
        self.torch.cuda.synchronize()

    def _entries(self, r):
        k = self._key(r)
        if k not in self.entries_per_view:
            self.entries_per_view[k] = 4 * self.scenes[r.scene].n
        return self.entries_per_view[k]

    def bytes_needed(self, r):
        n = self.scenes[r.scene].n
        ent = self._entries(r) * self.headroom
        # footprints (40 B/particle), entries with ping-pong (24 B), image + state (20 B/px)
        return int(40 * n + 24 * ent + 20 * r.pixels)

    def submit(self, batch):
        torch = self.torch
        si = self.busy.index(False)
        self.busy[si] = True
        s = self.streams[si]
        R = self.rasters[si]
        cams = [r.cam for r in batch]
        scenes = [self.scenes[r.scene] for r in batch]
        npv = [g.n for g in scenes]
        cap = int(sum(self._entries(r) for r in batch) * self.headroom) + 4096
        ev0 = None
        if self.record_spans:
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(s)
        with torch.cuda.stream(s):
            fp = R.project(scenes, cams)
            bins = R.bin_sort(fp, npv, cams, check=False, capacity=cap)
            img, _, _ = R.render_fwd_ordered(fp, npv, bins, cams, wide=True, last=False)
            status = self.status_host[si]   # {count, status}
            status.copy_(bins.count.as_strided((2,), (1,)), non_blocking=True)
            ev = torch.cuda.Event(enable_timing=self.record_spans)
            ev.record(s)
        if self.record_spans:
            self.spans.append((si, ev0, ev))
        return dict(si=si, batch=batch, ev=ev, fp=fp, bins=bins, img=img, status=status, npv=npv, cams=cams,
                    scenes=scenes)

    def poll(self, h):
        return h["ev"].query()

    def finish(self, h):
        torch = self.torch
        from .rasterizer import split_images
        count, st = int(h["status"][0]), int(h["status"][1])
        R = self.rasters[h["si"]]
        img = h["img"]
        if st != 0:
            # entry capacity overflow: redo this batch with the exact count (rare)
            self.overflows += 1
            with torch.cuda.stream(self.streams[h["si"]]):
                bins = R.bin_sort(h["fp"], h["npv"], h["cams"], check=True,
                                  capacity=int(count * self.headroom) + 4096)
                img, _, _ = R.render_fwd_ordered(h["fp"], h["npv"], bins, h["cams"], wide=True, last=False)
            self.streams[h["si"]].synchronize()
        for r, im in zip(h["batch"], split_images(img, h["cams"])):
            r.result = im
        self.busy[h["si"]] = False

    def device_overlap(self):
        """From the recorded device spans (after the batches completed): the number of batch
        pairs on different streams whose spans intersect, the time with at least two batches
        on the device and the time with at least one (milliseconds)."""
        if not self.spans:
            return dict(batches=0, overlapping_pairs=0, overlap_ms=0.0, busy_ms=0.0)
        self.torch.cuda.synchronize()
        ref = self.spans[0][1]
        iv = [(si, ref.elapsed_time(a), ref.elapsed_time(b)) for si, a, b in self.spans]
        pairs = sum(1 for i in range(len(iv)) for j in range(i + 1, len(iv))
                    if iv[i][0] != iv[j][0] and iv[i][1] < iv[j][2] and iv[j][1] < iv[i][2])
        pts = sorted([(a, 1) for _, a, _ in iv] + [(b, -1) for _, _, b in iv])
        depth, last, two, one = 0, None, 0.0, 0.0
        for t, d in pts:
            if last is not None:
                two += (t - last) if depth >= 2 else 0.0
                one += (t - last) if depth >= 1 else 0.0
            depth += d
            last = t
        return dict(batches=len(iv), overlapping_pairs=pairs, overlap_ms=two, busy_ms=one)
