"""The serving loop's admission logic on a simulated clock (no GPU): slots
and the memory budget are never exceeded, the queue is first come first
served, reservations return when results are released, a request that can
never fit is rejected, and latency percentiles come out of the clock."""
import numpy as np
import pytest

from paper_1501_03545_amd import serve as S
from paper_1501_03545_amd import workloads as W


def _stream(k, gap, n=1000, deg=10.0):
    return [(i * gap, dict(n=n, avg_degree=deg, gamma=2.5, seed=i)) for i in range(k)]


def _replay(trace):
    """Requests in flight and reserved bytes over the simulated run."""
    inflight, peak = set(), 0
    for t, ev, rid in sorted(trace, key=lambda x: (x[0], {"done": 0, "release": 1, "launch": 2}[x[1]])):
        if ev == "launch":
            inflight.add(rid)
        elif ev == "done":
            inflight.discard(rid)
        peak = max(peak, len(inflight))
    return peak


def test_slots_bound_concurrency_and_queue_is_fifo():
    ex = S.SimExecutor(cost=lambda p: 0.010)
    srv = S.Server(ex, slots=4, budget_bytes=1e12, hold_s=0.5)
    st = srv.run(_stream(40, 0.0))  # a burst: everything arrives at t = 0
    assert st["requests"] == 40 and st["rejected"] == 0
    assert st["max_inflight"] == 4 and _replay(ex.trace) == 4
    order = [rid for _, _, rid in ex.launched]
    assert order == sorted(order)
    # 10 waves of 4 requests, 10 ms each
    assert st["wall_s"] == pytest.approx(0.100)
    assert st["p50_ms"] == pytest.approx(50.0) and st["p99_ms"] == pytest.approx(100.0)


def test_budget_bounds_reserved_memory_and_waits_for_release():
    one = S.expected_bytes(1000, 10.0)
    ex = S.SimExecutor(cost=lambda p: 0.001)
    srv = S.Server(ex, slots=16, budget_bytes=2.5 * one, hold_s=0.2)
    st = srv.run(_stream(6, 0.0))
    assert st["max_reserved_bytes"] <= 2.5 * one
    assert st["max_inflight"] == 2
    # pairs run back to back, each pair waiting for the previous one's release
    launches = [t for t, _, _ in ex.launched]
    assert launches == pytest.approx([0, 0, 0.201, 0.201, 0.402, 0.402])
    assert srv.reserved == 0  # everything released at the end


def test_oversized_request_is_rejected_not_stalled():
    ex = S.SimExecutor(cost=lambda p: 0.001)
    stream = _stream(3, 0.01)
    stream[1] = (0.01, dict(n=10_000_000, avg_degree=16.0, gamma=2.5, seed=9))
    srv = S.Server(ex, slots=2, budget_bytes=S.expected_bytes(1000, 10.0) * 4, hold_s=0.0)
    st = srv.run(stream)
    assert st["requests"] == 2 and st["rejected"] == 1 and srv.rejected[0].rid == 1


def test_poisson_stream_statistics():
    stream = W.serve_stream(duration_s=5.0, rate_hz=200.0, seed=5)
    gaps = np.diff([t for t, _ in stream])
    assert len(stream) == pytest.approx(1000, rel=0.1)
    assert gaps.mean() == pytest.approx(1 / 200.0, rel=0.1)
    large = sum(1 for _, p in stream if p["n"] == 10_000_000)
    assert 5 <= large <= 40
    # cost proportional to the work; the large requests dominate the tail
    ex = S.SimExecutor(cost=lambda p: 2e-9 * p["n"] * (4 + p["avg_degree"]) + 1e-4)
    srv = S.Server(ex, slots=16, budget_bytes=200e9, hold_s=1.0)
    st = srv.run(stream)
    assert st["requests"] == len(stream)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["p99_ms"] >= 1e3 * 2e-9 * 1e7 * 20 * 0.5
    assert st["edges"] == sum(int(p["n"] * p["avg_degree"] / 2) for _, p in stream)


def test_library_footprint_is_what_the_buffers_take():
    P = pytest.importorskip("paper_1501_03545_amd")
    for d in W.batch_params(count=24, seed=11) + [dict(n=0, avg_degree=3.0, gamma=2.5, seed=1)]:
        p = P.rhg_plan(d["n"], d["avg_degree"], d["gamma"], d["seed"])
        b = P.GraphBuffers(p, None, device="cpu")
        held = sum(t.numel() * t.element_size() for t in (b.r, b.theta, b.ws, b.row_ptr, b.col))
        assert S.library_footprint(p) == held, d
