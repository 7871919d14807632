"""Benchmark: random hyperbolic graph generation on one MI355X.

One step = the whole hot path over one graph: sample the points, build the
index (keys, radix sort, band starts, cell directory, sorted records),
count pass, scan, emit pass.  All device buffers are allocated before the
timed region; the emit call's 8-byte read of 2m is inside it.

Prints one JSON line (see the keys below).  `value` is undirected edges per
second of the whole job.  `roofline` is the dominant kernel's achieved
bandwidth (its algorithmic bytes per launch over its average launch time,
both measured with HIP events on the library's stream during the timed
steps).  `cpu_baseline` times the CPU oracle on a bounded sample of the same
workload and scales it to the full job.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "undirected edges/sec at n=1e8 on 1 MI355X (% HBM roofline); p50/p99 request latency"


def _source_sha() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1501_03545_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(phase: str, n: int, m: int) -> int:
    """Minimum bytes a phase must move per launch (stated in the design doc)."""
    if phase == "sample":
        return 16 * n                      # write r, theta
    if phase == "keys+sort":
        return 16 * n + 8 * n              # read r, theta; write sorted key + id
    if phase == "gather":
        return 4 * n + 16 * n + 16 * n     # read ids, gather r, theta; write sorted r, theta
    if phase == "count":
        return 16 * n + 8 * n              # read r, theta once; write row_ptr
    if phase == "scan":
        return 16 * n                      # read + write row_ptr
    if phase == "emit":
        return 16 * n + 8 * n + 8 * m      # read r, theta and row_ptr; write 2m int32
    return 0


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
    return dict(ms_per_step=(t1 - t0) * 1000.0 / steps, nnz=nnz, phases=phases, stats=stats,
                params=p)


def cpu_baseline(cfg, params, m_edges, sample_pts):
    """Oracle pair-test rate on all pairs among the first `sample_pts`
    points of the same graph, scaled to the oracle's full job
    (n samples + 2 n (n-1) ordered pair tests: degrees, then CSR fill)."""
    import oracle as O
    O.build(force=False)
    n = cfg["n"]
    t0 = time.perf_counter()
    r, t, _ = O.sample(cfg["seed"], params.alpha, params.R, sample_pts)
    t1 = time.perf_counter()
    O.degrees(r, t, params.R)
    t2 = time.perf_counter()
    per_pt = (t1 - t0) / sample_pts
    rate = sample_pts * (sample_pts - 1) / (t2 - t1)  # ordered pair tests per second
    full_s = n * per_pt + 2.0 * n * (n - 1) / rate
    return {"value": m_edges / full_s, "unit": "undirected edges/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": "all %d ordered pair tests among the first %d points of the same graph "
                      "(+ sampling them), %.1f s wall; scaled to the full job of %d samples and "
                      "2n(n-1) pair tests = %.3g s" % (sample_pts * (sample_pts - 1), sample_pts,
                                                      t2 - t0, n, full_s)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--cpu-sample", type=int, default=60_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--band-width", type=float, default=0.0)
    ap.add_argument("--cell-target", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    from paper_1501_03545_amd import workloads as W
    cfg = W.SINGLE[args.config]
    tuning = None
    if args.band_width or args.cell_target:
        tuning = {"band_width": args.band_width, "cell_target": args.cell_target}
    res = run_gpu(cfg, args.steps, args.warmup, tuning)
    n = cfg["n"]
    m = res["nnz"] // 2
    sec = res["ms_per_step"] / 1000.0
    phases = res["phases"]
    dom = max(phases, key=lambda k: phases[k][0])
    dom_ms = phases[dom][0]
    achieved = algorithmic_bytes(dom, n, m) / (dom_ms / 1000.0) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (dom, args.config))
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("source_sha") == _source_sha():
            traffic = t.get("bytes_per_launch")
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
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": algorithmic_bytes(dom, n, m), "avg_launch_ms": dom_ms},
        "phases_ms": {k: round(v[0], 4) for k, v in phases.items()},
        "pipeline_floor_frac": (56 * n + 8 * m) / sec / 1e9 / HBM_PEAK_GBS,
        "search_stats": res["stats"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, res["params"], m, min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
