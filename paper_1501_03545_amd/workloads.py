"""Seeded synthetic workloads (the paper's own model: no dataset is needed).

This module holds parameter draws only; it carries none of the generator's
arithmetic, so the library, the oracle, the tests and the benchmark can all
use it.  The generator's inputs are (n, average degree, gamma, seed).
"""
from __future__ import annotations

import numpy as np

# single graphs: (n, target average degree, gamma, seed)
SMALL = dict(n=10_000, avg_degree=6.0, gamma=3.0, seed=1)         # oracle-sized
MEDIUM = dict(n=1_000_000, avg_degree=10.0, gamma=2.7, seed=2)    # FP64 search
LARGE = dict(n=100_000_000, avg_degree=20.0, gamma=2.2, seed=3)   # headline
SERVE_LARGE = dict(n=10_000_000, avg_degree=16.0, gamma=2.5)      # 2 % of requests

SINGLE = {"small": SMALL, "medium": MEDIUM, "large": LARGE}


def batch_params(count: int = 512, seed: int = 4):
    """Mixed batch: n log-uniform in [1e3, 1e6], average degree uniform in
    [4, 64], gamma uniform in [2.1, 3.5], per-graph seeds 0x5EED0000 + g.
    Draws are taken per graph in the order (u_n, u_k, u_gamma)."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(count):
        un, uk, ug = rng.random(3)
        out.append(dict(n=int(round(10 ** (3 + 3 * un))), avg_degree=4.0 + 60.0 * uk,
                        gamma=2.1 + 1.4 * ug, seed=0x5EED0000 + g))
    return out


def serve_stream(duration_s: float = 60.0, rate_hz: float = 200.0, seed: int = 5,
                 large_frac: float = 0.02):
    """Poisson arrivals: list of (arrival time in s, request params).  98 % of
    requests follow the batch distribution, 2 % are the large request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    k = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        if rng.random() < large_frac:
            p = dict(SERVE_LARGE)
        else:
            un, uk, ug = rng.random(3)
            p = dict(n=int(round(10 ** (3 + 3 * un))), avg_degree=4.0 + 60.0 * uk,
                     gamma=2.1 + 1.4 * ug)
        p["seed"] = 0x5E4E0000 + k
        out.append((t, p))
        k += 1
    return out


def move_batch(rng, r, theta, k: int, R: float, angle_step: float = 0.01, radius_step: float = 0.05):
    """k distinct vertices drawn uniformly; each drifts in angle by
    U(-angle_step, angle_step) (wrapped into [0, 2 pi)) and in radius by
    U(-radius_step, radius_step) (clipped into [0, R]).  numpy in, numpy out:
    (ids int32, new r, new theta)."""
    n = r.shape[0]
    ids = rng.choice(n, size=k, replace=False).astype(np.int32)
    t = theta[ids] + rng.uniform(-angle_step, angle_step, size=k)
    t = np.mod(t, 2 * np.pi)
    t = np.where(t >= 6.283185307179586, 0.0, t)
    rr = np.clip(r[ids] + rng.uniform(-radius_step, radius_step, size=k), 0.0, R)
    return ids, rr, t
