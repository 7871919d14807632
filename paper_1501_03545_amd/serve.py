"""Request loop for graph generation: continuous batching on one GPU.

Requests (n, average degree, gamma, seed) arrive over time.  The server keeps
up to `slots` requests in flight, each on its own HIP stream, so the work of
different requests overlaps on the device.  The queue is served first come
first served: its head is admitted as soon as a slot is free and its expected
device memory fits in the budget beside what is already reserved.  A request
reserves its points, its index workspace, its row offsets and the col_idx
slots of its expected edge count (the target degree times n, with slack);
the reservation is returned when the result is released, `hold_s` after it
completed (results stay on the device until then).  A request that could not
fit even into an empty budget is rejected at arrival.

Completion is observed by polling the HIP event recorded after the request's
last kernel; latency runs from arrival to that observation.  The executor is
pluggable: GpuExecutor drives the HIP library, SimExecutor replays the same
admission logic on a simulated clock for CPU tests.
"""
from __future__ import annotations

import collections
import heapq
import math
import time
from dataclasses import dataclass


@dataclass
class Request:
    rid: int
    arrival: float
    params: dict
    expected_bytes: int = 0
    admitted: float = -1.0
    done: float = -1.0
    edges: int = 0
    slot: int = -1
    result: object = None


def expected_bytes(n: int, avg_degree: float, slack: float = 1.3) -> int:
    """A size model of a request's device memory for the simulated executor:
    16 B per point for (r, theta), 64 B per point of index workspace, 8 B per
    row offset and 4 B per col_idx slot for n * avg_degree * slack directed
    edges."""
    return int(n * (16 + 64 + 8) + 8 + 4 * (int(n * avg_degree * slack) + 4096))


def library_footprint(params, tuning=None) -> int:
    """Device bytes of a request's buffers (GraphBuffers): (r, theta), the
    index workspace the library asks for, row_ptr and the col_idx slots
    reserved for the expected edge count.  Host-only query, no GPU work."""
    import paper_1501_03545_amd as P
    n = max(int(params.n), 1)
    return (16 * n + P.rhg_index_workspace_bytes(params, tuning) + 8 * (int(params.n) + 1)
            + 4 * max(P.expected_col_capacity(params), 1))


class Server:
    def __init__(self, executor, slots: int = 16, budget_bytes: float = 200e9, hold_s: float = 1.0,
                 keep=()):
        self.ex = executor
        self.slots = slots
        self.budget = budget_bytes
        self.hold_s = hold_s
        self.keep = set(keep)                # request ids whose results are handed to the caller
        self.reserved = 0
        self.free_slots = list(range(slots - 1, -1, -1))
        self.queue = collections.deque()     # arrived, not yet admitted
        self.inflight = {}                   # slot -> Request
        self.holding = []                    # heap of (release time, rid, Request)
        self.done = []
        self.rejected = []
        self.kept = {}
        self.max_reserved = 0
        self.max_inflight = 0
        self.busy_area = 0.0                 # integral of (requests in flight) dt
        self._last = None

    def _admit(self, now):
        while self.queue and self.free_slots:
            req = self.queue[0]
            if self.reserved + req.expected_bytes > self.budget:
                break  # first come first served: the head waits for memory
            self.queue.popleft()
            req.slot = self.free_slots.pop()
            req.admitted = now
            self.reserved += req.expected_bytes
            self.max_reserved = max(self.max_reserved, self.reserved)
            self.ex.launch(req.slot, req)
            self.inflight[req.slot] = req
        self.max_inflight = max(self.max_inflight, len(self.inflight))

    def _poll(self):
        for slot, req in list(self.inflight.items()):
            if self.ex.finished(slot, req):
                req.done = self.ex.now()
                req.edges = self.ex.edges(slot, req)
                del self.inflight[slot]
                self.free_slots.append(slot)
                self.done.append(req)
                heapq.heappush(self.holding, (req.done + self.hold_s, req.rid, req))
                if req.rid in self.keep:
                    self.kept[req.rid] = self.ex.take(req)

    def _release(self, until):
        while self.holding and self.holding[0][0] <= until:
            _, _, req = heapq.heappop(self.holding)
            self.ex.release(req)
            self.reserved -= req.expected_bytes

    def run(self, stream, poll_sleep: float = 2e-5):
        """stream: list of (arrival time in s, params dict), sorted by time.
        Returns the statistics of the run; results still held at the end are
        released."""
        pending = collections.deque(Request(i, t, p) for i, (t, p) in enumerate(stream))
        t0 = self.ex.now()
        self._last = t0
        while pending or self.queue or self.inflight:
            now_abs = self.ex.now()
            self.busy_area += len(self.inflight) * (now_abs - self._last)
            self._last = now_abs
            now = now_abs - t0
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                req.expected_bytes = self.ex.footprint(req)
                if req.expected_bytes > self.budget:
                    self.rejected.append(req)
                else:
                    self.queue.append(req)
            self._poll()
            self._release(self.ex.now())
            self._admit(now)
            if not (pending or self.queue or self.inflight):
                break
            events = []
            if pending:
                events.append(t0 + pending[0].arrival)
            if self.holding and self.queue:
                events.append(self.holding[0][0])
            self.ex.idle(poll_sleep, min(events) if events else None)
        wall = self.ex.now() - t0
        self._release(float("inf"))
        return self.stats(wall, t0)

    def stats(self, wall, t0):
        lat = sorted((r.done - t0) - r.arrival for r in self.done)

        def q(f):
            return lat[min(len(lat) - 1, max(0, int(math.ceil(f * len(lat))) - 1))] if lat else float("nan")

        edges = sum(r.edges for r in self.done)
        return {"requests": len(self.done), "rejected": len(self.rejected), "wall_s": wall,
                "p50_ms": q(0.50) * 1e3, "p99_ms": q(0.99) * 1e3,
                "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else float("nan"),
                "edges": edges, "edges_per_s": edges / wall if wall > 0 else 0.0,
                "max_reserved_bytes": self.max_reserved, "slots": self.slots,
                "max_inflight": self.max_inflight,
                "mean_inflight": self.busy_area / wall if wall > 0 else 0.0}


class GpuExecutor:
    """Runs each request's whole pipeline (rhg_generate_async, which neither
    allocates nor synchronises) on its slot's stream.  Buffers come from
    torch's caching allocator on that stream; 2m and the overflow flag come
    back through pinned host memory behind the request's completion event.
    A request whose edges overflow its reserved col_idx is emitted again into
    an exact buffer before it counts as complete."""

    def __init__(self, slots: int, tuning_fn=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.tuning_fn = tuning_fn
        self.plans = {}
        self.state = {}
        self.retries = 0

    def now(self):
        return time.perf_counter()

    def _submit(self, slot, rid, params, tuning, buf):
        import paper_1501_03545_amd as P
        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            flag = torch.empty(1, dtype=torch.int32, device=self.device)
            P.rhg_generate_async(params, buf.r, buf.theta, buf.ws, buf.row_ptr, buf.col, flag, tuning, s)
            tail = torch.stack([buf.row_ptr[-1], flag[0].to(torch.int64)])
            host = torch.empty(2, dtype=torch.int64, pin_memory=True)
            host.copy_(tail, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.state[rid] = (buf, host, ev, params, tuning)

    def footprint(self, req):
        """Plans the request at arrival (host only) and returns its bytes."""
        import paper_1501_03545_amd as P
        p = req.params
        params = P.rhg_plan(p["n"], p["avg_degree"], p["gamma"], p["seed"])
        tuning = self.tuning_fn(p["n"], p["avg_degree"], p["gamma"]) if self.tuning_fn else None
        self.plans[req.rid] = (params, tuning)
        return library_footprint(params, tuning)

    def launch(self, slot, req):
        import paper_1501_03545_amd as P
        params, tuning = self.plans.pop(req.rid)
        with self.torch.cuda.stream(self.streams[slot]):
            buf = P.GraphBuffers(params, tuning, device=self.device)
        self._submit(slot, req.rid, params, tuning, buf)

    def finished(self, slot, req):
        buf, host, ev, params, tuning = self.state[req.rid]
        if not ev.query():
            return False
        if int(host[1]) & 2:
            import paper_1501_03545_amd as P
            raise P.RhgError(P.RHG_EINTERNAL, "request %d: emit pass disagreed with the count pass" % req.rid)
        if int(host[1]) != 0:
            self.retries += 1
            with self.torch.cuda.stream(self.streams[slot]):
                buf.col = self.torch.empty(int(host[0]), dtype=self.torch.int32, device=self.device)
            self._submit(slot, req.rid, params, tuning, buf)
            return False
        buf.ws = None  # the index is not part of the result
        return True

    def edges(self, slot, req):
        return int(self.state[req.rid][1][0]) // 2

    def take(self, req):
        """The finished graph (GraphBuffers) of a request, for the caller."""
        return self.state[req.rid][0]

    def release(self, req):
        self.state.pop(req.rid, None)

    def idle(self, sleep_s, next_event):
        if sleep_s > 0:
            time.sleep(sleep_s)


class SimExecutor:
    """CPU stand-in: a request completes cost(params) seconds after it is
    launched, on a simulated clock that idle() advances to the next event."""

    def __init__(self, cost):
        self.cost = cost
        self.clock = 0.0
        self.finish = {}
        self.launched = []
        self.released = []
        self.trace = []  # (time, event, rid)

    def now(self):
        return self.clock

    def footprint(self, req):
        return expected_bytes(req.params["n"], req.params["avg_degree"])

    def launch(self, slot, req):
        self.finish[req.rid] = self.clock + self.cost(req.params)
        self.launched.append((self.clock, slot, req.rid))
        self.trace.append((self.clock, "launch", req.rid))

    def finished(self, slot, req):
        ok = self.finish[req.rid] <= self.clock
        if ok:
            self.trace.append((self.clock, "done", req.rid))
        return ok

    def edges(self, slot, req):
        return int(req.params["n"] * req.params["avg_degree"] / 2)

    def take(self, req):
        return req.rid

    def release(self, req):
        self.released.append((self.clock, req.rid))
        self.trace.append((self.clock, "release", req.rid))

    def idle(self, sleep_s, next_event):
        ev = [f for f in self.finish.values() if f > self.clock]
        if next_event is not None and next_event > self.clock:
            ev.append(next_event)
        self.clock = min(ev) if ev else self.clock + sleep_s


def run_native(server, stream, hold_s: float = 1.0, keep=(), poll_sleep: float = 2e-5, tuning_fn=None):
    """Drives the library's own server (RhgServer: admission, slots and
    device memory in native code) with a timed arrival stream: each request
    is submitted at its arrival time, completions are polled, and results are
    released hold_s after they completed (those in `keep` are handed back
    instead, as the completion dicts, for the caller to release).  Latency
    runs from arrival to the poll that saw the completion.  stream: list of
    (arrival time in s, params dict), sorted by time; arrival 0 for all gives
    the saturated server.  Returns (statistics, kept completions)."""
    import paper_1501_03545_amd as P
    keep = set(keep)
    pending = collections.deque(enumerate(stream))
    arrival = {}
    holding = []
    lat, kept = [], {}
    edges = 0
    rejected = failed = 0
    t0 = time.perf_counter()
    busy_area, last = 0.0, t0
    outstanding = 0
    while pending or outstanding:
        now = time.perf_counter()
        st = server.stats()
        busy_area += st["inflight"] * (now - last)
        last = now
        while pending and pending[0][1][0] <= now - t0:
            rid, (t, p) = pending.popleft()
            tun = tuning_fn(p["n"], p["avg_degree"], p["gamma"]) if tuning_fn else None
            try:
                server.submit(rid, p["n"], p["avg_degree"], p["gamma"], p["seed"], tun)
            except P.RhgError as e:
                if e.status != P.RHG_ECAPACITY:
                    raise
                rejected += 1
                continue
            arrival[rid] = t0 + t
            outstanding += 1
        for c in server.poll():
            rid = c["req_id"]
            done = time.perf_counter()
            outstanding -= 1
            if c["status"] != P.RHG_OK:
                failed += 1
                server.release(rid)
                continue
            lat.append(done - arrival.pop(rid))
            edges += c["nnz"] // 2
            if rid in keep:
                kept[rid] = c
            else:
                heapq.heappush(holding, (done + hold_s, rid))
        now = time.perf_counter()
        while holding and holding[0][0] <= now:
            server.release(heapq.heappop(holding)[1])
        if poll_sleep > 0 and (pending or outstanding):
            time.sleep(poll_sleep)
    wall = time.perf_counter() - t0
    while holding:
        server.release(heapq.heappop(holding)[1])
    lat.sort()

    def q(f):
        return lat[min(len(lat) - 1, max(0, int(math.ceil(f * len(lat))) - 1))] * 1e3 if lat else float("nan")

    st = server.stats()
    return ({"requests": len(lat), "rejected": rejected, "failed": failed, "wall_s": wall,
             "p50_ms": q(0.50), "p99_ms": q(0.99), "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else float("nan"),
             "edges": edges, "edges_per_s": edges / wall if wall > 0 else 0.0,
             "max_reserved_bytes": st["max_reserved_bytes"], "max_inflight": st["max_inflight"],
             "mean_inflight": busy_area / wall if wall > 0 else 0.0, "refills": st["refills"]}, kept)


def run_plain_loop(stream, device="cuda"):
    """The same requests as a plain loop: one graph after another on one
    stream (rhg_generate_async into freshly allocated buffers, a graph whose
    edges overflow its slots run again into exactly 2m), each result freed
    once the next graph is queued.  Returns (edges, wall seconds)."""
    import torch
    import paper_1501_03545_amd as P
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges = 0
    flags = []
    for i, (_, p) in enumerate(stream):
        params = P.rhg_plan(p["n"], p["avg_degree"], p["gamma"], p["seed"])
        b = P.GraphBuffers(params, device=device)
        flag = torch.zeros(1, dtype=torch.int32, device=device)
        P.rhg_generate_async(params, b.r, b.theta, b.ws, b.row_ptr, b.col, flag, None, s)
        flags.append((flag, b.row_ptr[-1:], params))
    torch.cuda.synchronize()
    for flag, tail, params in flags:
        if int(flag.item()):  # rare: run again with exact capacity
            b = P.GraphBuffers(params, col_capacity=int(tail.item()), device=device)
            f2 = torch.zeros(1, dtype=torch.int32, device=device)
            P.rhg_generate_async(params, b.r, b.theta, b.ws, b.row_ptr, b.col, f2, None, s)
        edges += int(tail.item()) // 2
    torch.cuda.synchronize()
    return edges, time.perf_counter() - t0
