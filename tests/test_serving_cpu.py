"""Scheduler logic of the serving loop on the CPU: a simulated executor on a virtual clock
(no GPU). Checks admission by memory, FIFO order, continuous batching (requests arriving
while batches run join later batches and batches overlap), and the latency statistics."""
import math

import numpy as np
import pytest

from paper_2403_14244_amd.serving import Request, Server, SimulatedExecutor, VirtualClock
import scenegen as S


def trace(n=400, rate=200.0, seed=4, res=((512, 512), (1280, 720), (1920, 1080))):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        w, h = res[int(rng.integers(len(res)))]
        out.append(Request(rid=i, scene=["a", "b"][int(rng.integers(2))],
                           cam=S.orbit_camera(float(rng.uniform(0, 2 * math.pi)), 4.0, w, h), arrival=t))
    return out


def run(reqs, pool, **kw):
    clock = VirtualClock()
    ex = SimulatedExecutor(clock, {"a": 200_000, "b": 1_000_000}, **{k: v for k, v in kw.items() if k in ("base", "per_mpix")})
    srv = Server(ex, pool_bytes=pool, clock=clock, max_batch=kw.get("max_batch", 16),
                 max_inflight=kw.get("max_inflight", 2))
    return srv, srv.run(reqs)


def test_every_request_completes_after_it_arrives_and_fifo_admission():
    reqs = trace()
    srv, st = run(reqs, pool=2 << 30)
    assert st["requests"] == len(reqs)
    assert all(r.done >= r.submit >= r.arrival for r in reqs)
    # admission is first come first served: submit times never decrease with arrival order
    order = sorted(reqs, key=lambda r: (r.arrival, r.rid))
    subs = [r.submit for r in order]
    assert all(b >= a for a, b in zip(subs, subs[1:]))


def test_memory_admission_never_exceeds_the_pool():
    reqs = trace(300, rate=2000.0)
    ex_bytes = max(40 * 1_000_000 + 20 * 1920 * 1080, 1)
    pool = 3 * ex_bytes                                  # at most ~3 large requests in flight
    srv, st = run(reqs, pool=pool, per_mpix=2e-3)
    assert st["peak_pool_bytes"] <= pool
    assert max(b[2] for b in srv.batches) <= pool
    assert st["requests"] == 300


def test_request_larger_than_pool_is_rejected():
    reqs = trace(5)
    with pytest.raises(ValueError):
        run(reqs, pool=1000)


def test_continuous_batching_overlaps_batches_and_admits_late_arrivals():
    """Under load, a request that arrives while a batch runs is admitted before that batch
    completes (into a second slot), so batches overlap in time."""
    reqs = trace(300, rate=3000.0)
    srv, st = run(reqs, pool=8 << 30, per_mpix=5e-4, max_inflight=2)
    by_batch = {}
    for r in reqs:
        by_batch.setdefault(r.batch, []).append(r)
    spans = sorted((min(r.submit for r in b), max(r.done for r in b)) for b in by_batch.values())
    overlaps = sum(1 for (s0, e0), (s1, e1) in zip(spans, spans[1:]) if s1 < e0)
    assert overlaps > 0.3 * len(spans)
    late = [r for r in reqs if any(s < r.arrival < e for s, e in spans) and r.submit < max(e for s, e in spans)]
    assert late
    assert st["mean_batch"] > 1.5


def test_single_slot_serialises_batches():
    reqs = trace(100, rate=3000.0)
    srv, st = run(reqs, pool=8 << 30, max_inflight=1)
    by_batch = {}
    for r in reqs:
        by_batch.setdefault(r.batch, []).append(r)
    spans = sorted((min(r.submit for r in b), max(r.done for r in b)) for b in by_batch.values())
    assert all(s1 >= e0 for (s0, e0), (s1, e1) in zip(spans, spans[1:]))


def test_latency_statistics():
    reqs = trace(200, rate=100.0)
    srv, st = run(reqs, pool=8 << 30, base=1e-3, per_mpix=0.0)
    lat = np.array([r.latency for r in reqs]) * 1e3
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    # at light load each request waits only for its own batch (1 ms) or one running batch
    assert st["p50_ms"] <= 2.0 + 1e-9 and st["p99_ms"] <= 2.0 + 1e-9
    assert set(st["p99_ms_by_resolution"]) == {"512x512", "1280x720", "1920x1080"}
