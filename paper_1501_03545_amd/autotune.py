"""Autotuner for the index and search tuning (band width, cell size, heavy
set) per class of graph.

A class is (size decade of n, gamma below/above 2.5, average degree below/
above 20).  For each class the tuner generates a representative graph and
times the whole pipeline (rhg_generate_async, HIP events on one stream) for
every candidate tuning, keeping the fastest.  The edge set does not depend
on the tuning, only the speed; results are cached per device in
tuning_cache.json next to this file.

    python -m paper_1501_03545_amd.autotune [copy.json]   # on a GPU: writes the cache
"""
from __future__ import annotations

import itertools
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

CANDIDATES = [dict(band_width=bw, cell_target=ct, heavy_points=hp)
              for bw, ct, hp in itertools.product([1.0, 1.5, 2.0, 3.0], [1, 4], [2048, 16384, 65536])]


def class_of(n: int, avg_degree: float, gamma: float) -> str:
    dec = int(min(7, max(3, round(math.log10(max(n, 10))))))
    return "n1e%d_g%s_k%s" % (dec, "lo" if gamma < 2.5 else "hi", "lo" if avg_degree < 20 else "hi")


def representative(cls: str):
    dec = int(cls[3])
    g = 2.3 if "_glo" in cls else 3.0
    k = 10.0 if "_klo" in cls else 40.0
    return 10 ** dec, k, g


_cache = None


def load_cache():
    global _cache
    if _cache is None:
        _cache = json.load(open(CACHE)) if os.path.exists(CACHE) else {}
    return _cache


def device_key() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def tuning_for(n: int, avg_degree: float, gamma: float):
    """The cached tuning of this graph's class on this device (None: library
    defaults)."""
    table = load_cache().get(device_key(), {})
    return table.get(class_of(n, avg_degree, gamma))


def time_tuning(n, k, g, tuning, reps=3):
    import torch
    import paper_1501_03545_amd as P
    p = P.rhg_plan(n, k, g, 12345)
    buf = P.GraphBuffers(p, tuning, col_capacity=P.expected_col_capacity(p, 1.6))
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    P.rhg_generate_async(p, buf.r, buf.theta, buf.ws, buf.row_ptr, buf.col, flag, tuning, s)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        P.rhg_generate_async(p, buf.r, buf.theta, buf.ws, buf.row_ptr, buf.col, flag, tuning, s)
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b))
    assert int(flag.item()) == 0
    return sorted(times)[len(times) // 2]


def tune(classes=None, verbose=True):
    classes = classes or [class_of(10 ** d, k, g) for d in (3, 4, 5, 6, 7) for g in (2.3, 3.0) for k in (10.0, 40.0)]
    table = {}
    for cls in classes:
        n, k, g = representative(cls)
        best = None
        for cand in CANDIDATES:
            ms = time_tuning(n, k, g, cand)
            if best is None or ms < best[0]:
                best = (ms, cand)
        table[cls] = dict(best[1], ms=round(best[0], 4))
        if verbose:
            print(cls, table[cls], flush=True)
    cache = load_cache()
    cache[device_key()] = table
    json.dump(cache, open(CACHE, "w"), indent=1, sort_keys=True)
    return table


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    tune()
    if len(sys.argv) > 1:  # also copy the cache to the given path
        import shutil
        shutil.copyfile(CACHE, sys.argv[1])
