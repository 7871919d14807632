"""Pins of the oracle's graph statistics: closed forms on small named graphs,
a brute-force triangle count, Pearson correlation computed directly, and the
power-law MLE on samples of a known exponent."""
import itertools
import math

import numpy as np

import oracle as O


def _csr(n, pairs):
    rows = [set() for _ in range(n)]
    for a, b in pairs:
        rows[a].add(b)
        rows[b].add(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in sorted(r)], dtype=np.int64)
    return rp, col


def test_named_graphs():
    n = 7
    s = O.graph_stats(*_csr(n, itertools.combinations(range(n), 2)), kmin=2)  # complete graph
    assert s["triangles"] == math.comb(n, 3) and s["transitivity"] == 1.0 and s["avg_local_clustering"] == 1.0
    assert math.isnan(s["assortativity"])  # regular: no degree variance
    assert s["hist"][3] == n  # degree 6 in [4, 8)
    s = O.graph_stats(*_csr(n, [(0, v) for v in range(1, n)]), kmin=2)  # star
    assert s["triangles"] == 0 and s["transitivity"] == 0.0 and s["assortativity"] == -1.0
    assert s["hist"][1] == n - 1 and s["hist"][3] == 1
    s = O.graph_stats(*_csr(n, [(v, (v + 1) % n) for v in range(n)]), kmin=2)  # cycle
    assert s["triangles"] == 0 and math.isnan(s["assortativity"])
    m = 9  # wheel: hub 0 and a cycle of m vertices
    pairs = [(0, v) for v in range(1, m + 1)] + [(v, v % m + 1) for v in range(1, m + 1)]
    s = O.graph_stats(*_csr(m + 1, pairs), kmin=2)
    assert s["triangles"] == m
    assert s["triads"] == m * (m - 1) // 2 + 3 * m
    assert s["transitivity"] == 3 * m / (m * (m - 1) / 2 + 3 * m)
    assert s["avg_local_clustering"] == (m * (2 / 3) + m / math.comb(m, 2)) / (m + 1)
    s = O.graph_stats(*_csr(4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]), kmin=2)  # diamond
    assert s["triangles"] == 2 and list(s["vertex_triangles"]) == [1, 2, 2, 1]


def test_triangles_and_correlation_by_brute_force():
    rng = np.random.default_rng(3)
    n = 60
    pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.15]
    rp, col = _csr(n, pairs)
    adj = np.zeros((n, n), dtype=bool)
    for a, b in pairs:
        adj[a, b] = adj[b, a] = True
    tri = sum(1 for a, b, c in itertools.combinations(range(n), 3) if adj[a, b] and adj[b, c] and adj[a, c])
    s = O.graph_stats(rp, col, kmin=3)
    assert s["triangles"] == tri
    deg = adj.sum(axis=1)
    x = np.array([deg[a] for a, b in pairs] + [deg[b] for a, b in pairs], dtype=float)
    y = np.array([deg[b] for a, b in pairs] + [deg[a] for a, b in pairs], dtype=float)
    assert abs(s["assortativity"] - np.corrcoef(x, y)[0, 1]) < 1e-12
    ok = deg >= 2
    loc = [sum(1 for u, w in itertools.combinations(np.flatnonzero(adj[v]), 2) if adj[u, w]) / math.comb(int(deg[v]), 2)
           for v in range(n) if ok[v]]
    assert abs(s["avg_local_clustering"] - np.mean(loc)) < 1e-12


def test_power_law_mle_recovers_the_exponent():
    rng = np.random.default_rng(11)
    alpha, kmin, N = 2.5, 10, 200_000
    # discrete power law by the usual rounding of the continuous inverse CDF
    k = np.floor((kmin - 0.5) * (1 - rng.random(N)) ** (-1 / (alpha - 1)) + 0.5).astype(np.int64)
    # a graph is not needed for the estimator: a star forest with these degrees
    rp = np.concatenate([[0], np.cumsum(k)])
    col = np.zeros(int(rp[-1]), dtype=np.int64)  # the estimator reads degrees only
    s = O.graph_stats(rp, col, kmin=kmin, triangles=False)
    sigma = (alpha - 1) / math.sqrt(N)
    assert s["tail_count"] == N
    assert abs(s["gamma_mle"] - alpha) < 5 * sigma + 0.01
