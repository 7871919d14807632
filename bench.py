"""Benchmark: random hyperbolic graph generation on one MI355X.

One step = the whole hot path over one graph: sample the points, build the
index (keys, radix sort, band starts, cell directory, sorted records),
count pass, scan, emit pass.  All device buffers are allocated before the
timed region; the emit call's 8-byte read of 2m is inside it.

Prints one JSON line (see the keys below).  `value` is undirected edges per
second of the whole job.  `roofline` is the dominant kernel's achieved
bandwidth: the method's bytes of that pass (its share of the floor
56n + 8m + 8) per launch over its average launch time, both measured with HIP
events on the library's stream during the timed steps, with the HBM traffic
rocprofv3 counted for the same kernel.  `step_roofline` puts the whole step
against the same floor (floor fraction), against the counted traffic
(achieved fraction and amplification) and against a measured device copy.
`cpu_baseline` times the CPU oracle's pair loop on bounded samples of the
same workload and extrapolates to the full job.
"""
from __future__ import annotations

import argparse
import math
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# rocprofv3 HBM-traffic summaries per workload (profiles/): scaled FETCH_SIZE +
# WRITE_SIZE per launch and per step, with the hash of the kernel sources
TRAFFIC_FILES = {"large": "traffic_n1e8_avgdeg20_gamma2.2.json"}
METRIC = "undirected edges/sec at n=1e8 on 1 MI355X (% HBM roofline); p50/p99 request latency"


def _log(*a):
    """Progress lines on stderr (stdout carries only the JSON line)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def _source_sha() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1501_03545_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(phase: str, n: int, m: int) -> int:
    """The method's own bytes per launch of a phase: its share of the floor
    B_alg = 56n + 8m + 8 of one generation (write the points, read them to
    index, read them once to search, write the row offsets, write col_idx).
    Everything else a phase moves (sort passes, sorted copies, the index's
    records) is the design's traffic, reported under `traffic`."""
    table = {
        "sample": 16 * n,                 # write r, theta
        "keys+sort": 16 * n,              # read r, theta to index them
        "count": 16 * n + 8 * (n + 1),    # read the points once to search; row offsets
        "emit": 8 * m,                    # col_idx: 4 bytes x 2m entries
    }
    return int(table.get(phase, 0))


def run_gpu(cfg, steps, warmup, tuning=None):
    import torch
    import paper_1501_03545_amd as P

    n = cfg["n"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = P.rhg_plan(n, cfg["avg_degree"], cfg["gamma"], cfg["seed"])
    r = torch.empty(n, dtype=torch.float64, device=dev)
    th = torch.empty(n, dtype=torch.float64, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ws = torch.empty(P.rhg_index_workspace_bytes(p, tuning), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def count_only():
        P.rhg_sample_points(p, r, th, stream)
        idx = P.rhg_build_index(p, r, th, tuning=tuning, workspace=ws, validate=False, stream=stream)
        P.rhg_count_edges(idx, row_ptr, stream)
        return idx

    idx = count_only()
    nnz = int(row_ptr[n].item())
    idx.free()
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)

    def step():
        idx = count_only()
        P.rhg_emit_edges(idx, row_ptr, col[:nnz], stream=stream)
        idx.free()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    P.rhg_set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = P.rhg_phase_times()
    P.rhg_set_profiling(False)
    # diagnostics of one more pass (outside the timed region)
    idx = count_only()
    P.rhg_emit_edges(idx, row_ptr, col[:nnz], stream=stream)
    stats = P.rhg_index_stats(idx, stream)
    idx.free()
    # canonical rows, apart from the step: the row sort of the emitted CSR,
    # on freshly emitted (search-order) rows each time
    sort_ws = torch.empty(P.rhg_sort_rows_workspace_bytes(n, nnz), dtype=torch.uint8, device=dev)
    rows_ms = []
    for rep in range(2):
        if rep:
            idx = count_only()
            P.rhg_emit_edges(idx, row_ptr, col[:nnz], stream=stream)
            idx.free()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.rhg_sort_rows(row_ptr, col[:nnz], nnz=nnz, workspace=sort_ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        rows_ms.append(e0.elapsed_time(e1))
    # validation statistics of the canonical graph (the last row sort left
    # col ascending): degrees, power-law exponent, assortativity
    st_ws = torch.empty(P.rhg_graph_stats_workspace_bytes(n, nnz, False), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    vstats = P.rhg_graph_stats(row_ptr, col[:nnz], kmin=10.0, triangles=False, nnz=nnz, workspace=st_ws)
    vstats_ms = (time.perf_counter() - t_s) * 1e3
    del st_ws
    # long-range augmentation (RHG-LR) of the same graph: 0.5 % extra edges
    k_lr = P.long_range_count(nnz // 2)
    lr_ws = torch.empty(P.rhg_long_range_workspace_bytes(n, k_lr), dtype=torch.uint8, device=dev)
    lr_out = (torch.empty(n + 1, dtype=torch.int64, device=dev),
              torch.empty(nnz + 2 * k_lr, dtype=torch.int32, device=dev))
    lr_ms = []
    for rep in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, _, added = P.rhg_long_range(row_ptr, col[:nnz], k_lr, cfg["seed"], nnz=nnz, workspace=lr_ws, out=lr_out,
                                       stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        lr_ms.append(e0.elapsed_time(e1))
    lr = {"k": k_lr, "added": int(added.item()), "ms": min(lr_ms)}
    del lr_ws, lr_out
    validation = {"workload": "the n=%d graph above" % n, "ms": vstats_ms, "kmin": 10.0,
                  "gamma_mle": vstats["gamma_mle"], "assortativity": vstats["assortativity"],
                  "max_degree": vstats["max_degree"]}
    return dict(ms_per_step=(t1 - t0) * 1000.0 / steps, nnz=nnz, phases=phases, stats=stats,
                params=p, rows_ms=min(rows_ms), lr=lr, validation=validation)


def run_validation_triangles():
    """Full validation statistics with triangles on the n = 1e7 serving
    graph (canonical rows)."""
    import torch
    import paper_1501_03545_amd as P
    from paper_1501_03545_amd import workloads as W
    cfg = dict(W.SERVE_LARGE, seed=1)
    g = P.rhg_generate(cfg["n"], cfg["avg_degree"], cfg["gamma"], cfg["seed"], canonical_rows=True)
    nnz = int(g.row_ptr[-1].item())
    ws = torch.empty(P.rhg_graph_stats_workspace_bytes(cfg["n"], nnz, True), dtype=torch.uint8, device="cuda")
    best, s = None, None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = P.rhg_graph_stats(g.row_ptr, g.col_idx, kmin=10.0, triangles=True, nnz=nnz, workspace=ws)
        ms = (time.perf_counter() - t0) * 1e3
        best = ms if best is None else min(best, ms)
    return {"workload": "rhg n=%d avg_degree=%g gamma=%g seed=%d, canonical rows" % (
                cfg["n"], cfg["avg_degree"], cfg["gamma"], cfg["seed"]),
            "ms": best, "triangles": s["triangles"], "transitivity": s["transitivity"],
            "avg_local_clustering": s["avg_local_clustering"], "gamma_mle": s["gamma_mle"],
            "assortativity": s["assortativity"]}


def run_batch(count, reps, tuned=True, n_streams=64):
    """The batch workload: `count` uneven graphs as one captured launch
    (autotuned per class when a tuning cache exists), against the plain
    per-graph loop over the same graphs (one stream, default tuning,
    preallocated buffers), and against rhg_generate per graph (allocation
    and one 8-byte readback per graph).  Edges/s over the whole batch."""
    import torch
    import paper_1501_03545_amd as P
    from paper_1501_03545_amd import autotune as A
    from paper_1501_03545_amd import workloads as W

    draws = W.batch_params(count=count)
    plans = [P.rhg_plan(d["n"], d["avg_degree"], d["gamma"], d["seed"]) for d in draws]
    tunings = [A.tuning_for(d["n"], d["avg_degree"], d["gamma"]) if tuned else None for d in draws]
    bufs = [P.GraphBuffers(p, t) for p, t in zip(plans, tunings)]
    batch = P.Batch(bufs, n_streams=n_streams)
    stream = torch.cuda.current_stream()
    batch.launch(stream)
    torch.cuda.synchronize()
    fixed = batch.fix_overflows()
    torch.cuda.synchronize()
    m = sum(int(b.row_ptr[-1].item()) for b in bufs) // 2

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_batch = timed(lambda: batch.launch(stream))
    batch.destroy()
    tuned_names = sorted({A.class_of(d["n"], d["avg_degree"], d["gamma"]) for d, t in zip(draws, tunings) if t})
    del bufs, batch
    torch.cuda.empty_cache()
    # the plain loop: same library, one graph after another, default tuning
    plain = [P.GraphBuffers(p, None) for p in plans]
    flags = torch.zeros(count, dtype=torch.int32, device="cuda")

    def loop():
        for g, b in enumerate(plain):
            P.rhg_generate_async(b.params, b.r, b.theta, b.ws, b.row_ptr, b.col, flags[g:g + 1], None, stream)

    t_loop = timed(loop)
    assert int(flags.sum().item()) == 0 or fixed, "plain loop overflowed"
    m_loop = sum(int(b.row_ptr[-1].item()) for b in plain) // 2
    del plain
    torch.cuda.empty_cache()

    def gen_loop():
        for d in draws:
            P.rhg_generate(d["n"], d["avg_degree"], d["gamma"], d["seed"], stream=stream)

    t_gen = timed(gen_loop)
    torch.cuda.empty_cache()
    return {"workload": "%d graphs: n log-uniform in [1e3, 1e6], avg degree uniform in [4, 64], "
                        "gamma uniform in [2.1, 3.5], seeds 0x5EED0000 + g" % count,
            "graphs": count, "sum_n": sum(d["n"] for d in draws), "undirected_edges": m,
            "edges_match_plain_loop": m == m_loop,
            "batched": {"ms": t_batch * 1e3, "edges_per_s": m / t_batch, "streams": n_streams,
                        "form": "one captured HIP graph launch", "tuned_classes": tuned_names},
            "plain_loop": {"ms": t_loop * 1e3, "edges_per_s": m / t_loop,
                           "form": "rhg_generate_async per graph, one stream, default tuning"},
            "generate_loop": {"ms": t_gen * 1e3, "edges_per_s": m / t_gen,
                              "form": "rhg_generate per graph (allocates, reads back 2m)"},
            "speedup_vs_plain_loop": t_loop / t_batch, "overflow_refills": len(fixed), "reps": reps}


def run_serve(duration_s, rate_hz=200.0, slots=16, budget=200e9, hold_s=1.0, saturate=3000):
    """The serving workload on the library's own server (rhg_server_*:
    admission by its device arena, slots, device-resident results): Poisson
    arrivals at rate_hz for duration_s, results released hold_s after they
    complete.  Then the capacity run: the first `saturate` requests of the
    same stream all queued at once (each released as it completes), against
    the plain per-graph loop over the same requests."""
    import torch
    import paper_1501_03545_amd as P
    from paper_1501_03545_amd import autotune as A
    from paper_1501_03545_amd import serve as S
    from paper_1501_03545_amd import workloads as W

    srv = P.RhgServer(budget_bytes=int(budget), slots=slots)
    S.run_native(srv, W.serve_stream(duration_s=0.5, rate_hz=rate_hz, seed=99), hold_s=0.0, tuning_fn=A.tuning_for)
    stream = W.serve_stream(duration_s=duration_s, rate_hz=rate_hz, seed=5)
    st, _ = S.run_native(srv, stream, hold_s=hold_s, tuning_fn=A.tuning_for)
    offered = sum(p["n"] * p["avg_degree"] / 2 for _, p in stream) / duration_s
    st.update({"workload": "Poisson arrivals at %g req/s for %g s: 98%% drawn like the batch, 2%% at "
                           "n=1e7 avg degree 16 gamma 2.5" % (rate_hz, duration_s),
               "form": "rhg_server_* (native admission, %d slots, a %g GB device arena)" % (slots, budget / 1e9),
               "budget_bytes": budget, "hold_s": hold_s, "offered_edges_per_s": offered})
    burst = [(0.0, p) for _, p in stream[:saturate]]
    sat, _ = S.run_native(srv, burst, hold_s=0.0, tuning_fn=A.tuning_for)
    srv.close()
    del srv
    torch.cuda.empty_cache()
    edges, wall = S.run_plain_loop(burst)
    torch.cuda.empty_cache()
    sat.update({"workload": "the first %d requests of the stream above, all queued at once" % len(burst)})
    capacity = {"served": sat, "plain_loop": {"edges": edges, "wall_s": wall, "edges_per_s": edges / wall,
                                              "form": "rhg_generate_async per request, one stream"},
                "speedup_vs_plain_loop": sat["edges_per_s"] / (edges / wall)}
    return st, capacity


# Temperature model: the coins' Philox blocks bound the rate.  One coin is a
# Philox4x32-10 block: 10 rounds of two 32 x 32 -> 64-bit products (one
# v_mad_u64_u32 each) and four 32-bit xors, 60 vector instructions.  The
# chip issues 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 32-bit lane
# operations per second (the 157.3 TFLOP/s FP32 figure counts each as a
# packed pair of FMAs, 4 flops).
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
COIN_VALU_OPS = 60
COIN_PEAK_PER_S = VALU_LANE_OPS_PER_S / COIN_VALU_OPS


def run_temperature(cfg, T, reps=3, band_width=0.7, oracle_pts=40_000):
    """The temperature model on the single-graph workload: index once, then
    count + scan + emit passes timed with the library's phase events; the
    oracle's brute force timed on the first `oracle_pts` points."""
    import statistics
    import torch
    import paper_1501_03545_amd as P
    n = cfg["n"]
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    tuning = {"band_width": band_width}
    p = P.rhg_plan(n, cfg["avg_degree"], cfg["gamma"], cfg["seed"])
    r = torch.empty(n, dtype=torch.float64, device=dev)
    th = torch.empty(n, dtype=torch.float64, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    P.rhg_sample_points(p, r, th, stream)
    idx = P.rhg_build_index(p, r, th, tuning=tuning, validate=False, stream=stream)
    P.rhg_temp_count_edges(idx, T, row_ptr, stream)
    nnz = int(row_ptr[n].item())
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    P.rhg_temp_emit_edges(idx, T, row_ptr, col[:nnz], stream=stream)
    torch.cuda.synchronize()
    P.rhg_set_profiling(True)
    walls = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.rhg_temp_count_edges(idx, T, row_ptr, stream)
        P.rhg_temp_emit_edges(idx, T, row_ptr, col[:nnz], stream=stream)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
    phases = P.rhg_phase_times()
    P.rhg_set_profiling(False)
    st = P.rhg_index_stats(idx, stream)
    idx.free()
    del col
    torch.cuda.empty_cache()
    m = nnz // 2
    ms = statistics.median(walls)
    count_ms = phases["count"][0]
    coin_rate = st["temp_coins"] / (count_ms / 1e3)
    # the oracle: every pair with its coin, on the first oracle_pts points
    import oracle as O
    O.build(force=False)
    k = min(oracle_pts, n)
    ro, to, _ = O.sample(cfg["seed"], p.alpha, p.R, k, nthreads=O.threads())
    t0 = time.perf_counter()
    O.temp_csr(ro, to, p.R, T, cfg["seed"], nthreads=O.threads())
    o_s = time.perf_counter() - t0
    o_rate = k * (k - 1) / 2 / o_s
    return {"workload": "rhg n=%d avg_degree=%g gamma=%g seed=%d, temperature T=%g (Fermi-Dirac p(d), one Philox "
                        "coin per pair), band_width %g" % (n, cfg["avg_degree"], cfg["gamma"], cfg["seed"], T,
                                                           band_width),
            "undirected_edges": m, "ms_count_scan_emit": ms, "edges_per_s": m / (ms / 1e3),
            "phases_ms": {kk: round(v[0] * v[1] / reps, 4) for kk, v in phases.items() if v[1]},
            "candidates": st["temp_candidates"], "coins": st["temp_coins"], "fp32_undecided": st["fp32_undecided"],
            "dd_fallbacks": st["dd_fallbacks"], "ties": st["ties"],
            "roofline": {"bound": "alu", "kernel": "temp_kernel (count pass)", "achieved": coin_rate,
                         "peak": COIN_PEAK_PER_S, "unit": "coins/s", "frac": coin_rate / COIN_PEAK_PER_S,
                         "avg_launch_ms": count_ms,
                         "peak_basis": "Philox4x32-10 alone: 60 VALU instructions per coin (20 v_mad_u64_u32, "
                                       "40 v_xor_b32) at 256 CUs x 64 lanes x 2.4 GHz = 3.93e13 lane-ops/s"},
            "cpu_baseline": {"kind": "oracle", "cores": O.threads(),
                             "sample": "oracle temp_csr (every pair with its coin) over the first %d points: %.2f s"
                                       % (k, o_s),
                             "pairs_per_s": o_rate,
                             "value": m / (n * (n - 1) / 2 / o_rate), "unit": "undirected edges/s (extrapolated)"}}


def run_dynamic(cfg, regen_ms, moves=(10_000, 1_000_000), steps=4, angle_step=0.01, radius_step=0.05):
    """The dynamic model on the single-graph workload: the graph of the n
    sampled points is kept up to date while batches of k vertices move
    (each drifting by U(-0.01, 0.01) in angle and U(-0.05, 0.05) in radius,
    clipped to the disk); every step leaves the graph that regeneration
    from scratch with ascending rows would give.  regen_ms: that
    regeneration's time (one step of the main workload plus its row sort)."""
    import statistics
    import torch
    import paper_1501_03545_amd as P
    n = cfg["n"]
    dev = torch.device("cuda", 0)
    p = P.rhg_plan(n, cfg["avg_degree"], cfg["gamma"], cfg["seed"])
    r = torch.empty(n, dtype=torch.float64, device=dev)
    th = torch.empty(n, dtype=torch.float64, device=dev)
    P.rhg_sample_points(p, r, th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = P.DynGraph(p, r, th)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg["seed"] + 17)
    out = {"workload": "rhg n=%d avg_degree=%g gamma=%g seed=%d; per step k distinct vertices drift by U(-%g, %g) "
                       "in angle and U(-%g, %g) in radius (clipped to the disk)"
                       % (n, cfg["avg_degree"], cfg["gamma"], cfg["seed"], angle_step, angle_step, radius_step,
                          radius_step),
           "create_ms": create_ms, "regenerate_ms": regen_ms, "steps": []}
    for k in moves:
        k = min(k, n)
        times, changed, entries = [], [], []
        for _ in range(steps + 1):
            cur = d.graph()
            ids = torch.randperm(n, generator=gen, device=dev)[:k].to(torch.int32)
            rn = (cur.r[ids.long()] + (torch.rand(k, generator=gen, device=dev, dtype=torch.float64) * 2 - 1)
                  * radius_step).clamp_(0.0, p.R)
            tn = torch.remainder(cur.theta[ids.long()] + (torch.rand(k, generator=gen, device=dev,
                                                                     dtype=torch.float64) * 2 - 1) * angle_step,
                                 2 * math.pi)
            tn = torch.where(tn >= 6.283185307179586, torch.zeros_like(tn), tn)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d.move(ids, rn, tn)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            st = d.last_step()
            changed.append(st["changed_rows"])
            entries.append(st["moved_entries"])
        ms = statistics.median(times[1:])
        out["steps"].append({"k": k, "ms_per_step": ms, "moves_per_s": k / (ms / 1e3),
                             "changed_rows": int(statistics.median(changed[1:])),
                             "moved_rows_entries": int(statistics.median(entries[1:])),
                             "speedup_vs_regenerate": regen_ms / ms})
    nnz = d.graph().nnz
    d.close()
    # method's bytes of a step at these sizes: the index's sorted arrays read
    # and written (key, id, r, theta, FP32 record: 40 B a point), the row
    # offsets read and written (16 B a point) and every CSR entry read and
    # written (8 B an entry)
    alg = 96 * n + 8 * nnz
    out["roofline"] = {"bound": "hbm", "kernel": "rhg_dyn_move (whole step, k = %d)" % out["steps"][0]["k"],
                       "algorithmic_bytes": alg, "achieved": alg / (out["steps"][0]["ms_per_step"] / 1e3) / 1e9,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": alg / (out["steps"][0]["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS}
    return out


def copy_calibration(nbytes=4 << 30, reps=5):
    """A plain device-to-device copy of known size: its event-timed rate is
    the practical HBM ceiling, and under rocprofv3 --pmc its FETCH_SIZE and
    WRITE_SIZE per dispatch calibrate those counters (nbytes each way)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"bytes_each_way": nbytes, "ms": ms, "GB_s": 2 * nbytes / (ms / 1000.0) / 1e9}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, params, m_edges, all_pts=40_000, one_pts=10_000, reps=3):
    """The oracle's pair loop (every pair i < j tested once, the points
    already in memory), timed around the loop alone, median of `reps`: on
    all host threads over the first `all_pts` points of the graph, on one
    thread over the first `one_pts`, and the n = 1e4 graph in full.  `value`
    is the whole job's edges/s extrapolated from the all-core rate
    (n (n - 1) / 2 pairs)."""
    import statistics
    import oracle as O
    O.build(force=False)
    threads = O.threads()
    n = cfg["n"]
    r, t, _ = O.sample(cfg["seed"], params.alpha, params.R, all_pts, nthreads=threads)

    def rate(rr, tt, R, nt):
        secs = [O.pair_scan(rr, tt, R, nthreads=nt, timing=True)[-1] for _ in range(reps)]
        med = statistics.median(secs)
        k = rr.shape[0]
        return k * (k - 1) / 2 / med, med

    all_rate, all_s = rate(r, t, params.R, threads)
    one_rate, one_s = rate(r[:one_pts], t[:one_pts], params.R, 1)
    a1, R1 = O.solve_R(10_000, 6.0, 3.0)
    r1, t1, _ = O.sample(1, a1, R1, 10_000, nthreads=threads)
    c1_rate, c1_s = rate(r1, t1, R1, threads)
    O.threads()  # (the next oracle call sets its own thread count)
    full_s = n * (n - 1) / 2 / all_rate
    return {"value": m_edges / full_s, "unit": "undirected edges/s", "cores": threads, "kind": "oracle",
            "sample": "pair loop only (points preloaded), median of %d: all %d threads over the first %d points "
                      "of the same graph, %.3g pairs/s (%.2f s); one thread over the first %d points, %.3g pairs/s; "
                      "whole job extrapolated as n(n-1)/2 = %.3g pairs / the all-thread rate = %.3g s"
                      % (reps, threads, all_pts, all_rate, all_s, one_pts, one_rate, n * (n - 1) / 2, full_s),
            "pairs_per_s_all_threads": all_rate, "pairs_per_s_one_thread": one_rate,
            "c1_full": {"workload": "rhg n=10000 avg_degree=6 gamma=3 seed=1", "pair_loop_s": c1_s,
                        "pairs_per_s": c1_rate},
            "host": {"nproc": os.cpu_count(), "omp_threads": threads, "cpu_model": _cpu_model()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--cpu-sample", type=int, default=40_000, help="points of the all-thread oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=512, help="graphs in the batch workload (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving run (0: skip)")
    ap.add_argument("--band-width", type=float, default=0.0)
    ap.add_argument("--temperature", type=float, default=0.1, help="temperature-model leg at this T (0: skip)")
    ap.add_argument("--dynamic", type=int, default=1, help="dynamic-model leg (0: skip)")
    ap.add_argument("--cell-target", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    from paper_1501_03545_amd import workloads as W
    cfg = W.SINGLE[args.config]
    tuning = None
    if args.band_width or args.cell_target:
        tuning = {"band_width": args.band_width, "cell_target": args.cell_target}
    _log("single graph", cfg)
    res = run_gpu(cfg, args.steps, args.warmup, tuning)
    _log("single graph done: %.3f ms/step" % res["ms_per_step"])
    params = res["params"]
    n = cfg["n"]
    m = res["nnz"] // 2
    sec = res["ms_per_step"] / 1000.0
    phases = res["phases"]
    # the dominant kernel: the longer of the two search passes.  The count
    # phase brackets exactly the search kernel's launch on the library's
    # stream; after a staged count the emit phase brackets the emit pass's
    # launches (heavy chunks, the copy of the staged rows, the standby
    # re-search), otherwise the one emit search kernel.
    dom = max((k for k in ("count", "emit") if phases.get(k, (0, 0))[1]), key=lambda k: phases[k][0])
    dom_ms = phases[dom][0]
    alg = algorithmic_bytes(dom, n, m)
    achieved = alg / (dom_ms / 1000.0) / 1e9
    floor_bytes = 56 * n + 8 * m + 8
    _log("copy calibration")
    copy = copy_calibration()
    # HBM traffic from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
    # workload, taken on these very kernel sources (else null)
    traffic, step_bytes, prof_src = None, None, None
    tfile = os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(args.config, ""))
    if os.path.isfile(tfile):
        t = json.load(open(tfile))
        prof_src = t.get("source_sha")
        if prof_src == _source_sha():
            traffic = t.get("bytes_per_launch", {}).get(dom)
            step_bytes = t.get("step_bytes")
    step_gbs = step_bytes / sec / 1e9 if step_bytes else None
    step = {"floor_bytes": floor_bytes, "floor_frac": floor_bytes / sec / 1e9 / HBM_PEAK_GBS,
            "achieved_bytes": step_bytes, "achieved_GB_s": step_gbs,
            "achieved_frac": step_gbs / HBM_PEAK_GBS if step_gbs else None,
            "amplification": step_bytes / floor_bytes if step_bytes else None,
            "copy_GB_s": copy["GB_s"], "copy_frac": step_gbs / copy["GB_s"] if step_gbs else None,
            "traffic_source": os.path.relpath(tfile, ROOT) if traffic is not None else
            ("stale profile (sources changed since %s)" % prof_src if prof_src else None)}
    out = {
        "metric": METRIC,
        "value": m / sec,
        "unit": "undirected edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rhg n=%d avg_degree=%g gamma=%g seed=%d (%s graph)" % (
            n, cfg["avg_degree"], cfg["gamma"], cfg["seed"], args.config),
            "n": n, "avg_degree": cfg["avg_degree"], "gamma": cfg["gamma"], "R": res["params"].R,
            "undirected_edges": m, "parallelism": "1 gpu"},
        "roofline": {"bound": "hbm", "kernel": "search_kernel (%s pass)" % dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": alg, "avg_launch_ms": dom_ms,
                     "traffic_frac": traffic / (dom_ms / 1000.0) / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "amplification": traffic / alg if traffic else None},
        "step_roofline": step,
        "phases_ms": {k: round(v[0] * v[1] / args.steps, 4) for k, v in phases.items() if v[1]},
        "canonical_rows": {"ms": res["rows_ms"], "form": "rhg_sort_rows on the emitted CSR (ascending rows), "
                           "timed apart from the step and not in value"},
        "long_range": dict(res["lr"], form="rhg_long_range: ceil(0.005 m) random extra edges merged into the "
                           "emitted CSR (RHG-LR), timed apart from the step and not in value"),
        "validation": res["validation"],
        "search_stats": res["stats"],
        "copy_calibration": copy,
    }
    _log("validation statistics with triangles (n=1e7)")
    out["validation_triangles"] = run_validation_triangles()
    if args.temperature > 0:
        import torch
        del res
        torch.cuda.empty_cache()
        _log("temperature model, T =", args.temperature)
        out["temperature"] = run_temperature(cfg, args.temperature)
        _log("temperature done: %.2f ms, %.3g edges/s" % (out["temperature"]["ms_count_scan_emit"],
                                                          out["temperature"]["edges_per_s"]))
    if args.dynamic:
        import torch
        torch.cuda.empty_cache()
        _log("dynamic model")
        out["dynamic"] = run_dynamic(cfg, out["ms_per_step"] + out["canonical_rows"]["ms"])
        _log("dynamic done: %s" % ", ".join("k=%d %.2f ms" % (x["k"], x["ms_per_step"]) for x in out["dynamic"]["steps"]))
    if args.batch > 0:
        import torch
        torch.cuda.empty_cache()
        _log("batch of", args.batch)
        out["batch"] = run_batch(args.batch, args.batch_reps)
        _log("batch done: %.2f ms batched, %.2f ms plain loop" % (out["batch"]["batched"]["ms"],
                                                                  out["batch"]["plain_loop"]["ms"]))
    if args.serve_seconds > 0:
        _log("serving for %g s" % args.serve_seconds)
        out["serve"], out["serve_capacity"] = run_serve(args.serve_seconds)
        _log("serve done: p50 %.2f ms p99 %.2f ms; saturated %.3g edges/s vs plain loop %.3g" % (
            out["serve"]["p50_ms"], out["serve"]["p99_ms"], out["serve_capacity"]["served"]["edges_per_s"],
            out["serve_capacity"]["plain_loop"]["edges_per_s"]))
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg, params, m, all_pts=min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
