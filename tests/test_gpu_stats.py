"""Validation statistics on the GPU (rhg_graph_stats through the C ABI)
against the oracle's numpy/scipy definitions: integer results (histogram,
maximum and tail counts, triads, triangles) exactly, floating results
within a relative 1e-9 (sums of up to ~10^6 binary64 terms in another
order: n * 2^-53 is about 1e-10).  Also: the same bits on every run, the
ascending-row requirement of the triangle count, degenerate graphs."""
import itertools
import math
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P

pytestmark = pytest.mark.gpu

REL = 1e-9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _dev(rp, col):
    import torch
    return (torch.from_numpy(np.asarray(rp, dtype=np.int64)).cuda(),
            torch.from_numpy(np.asarray(col, dtype=np.int32)).cuda())


def _close(a, b):
    if math.isnan(b):
        return math.isnan(a)
    return abs(a - b) <= REL * max(1.0, abs(b))


def _compare(rp, col, kmin=3.0):
    g = P.rhg_graph_stats(*_dev(rp, col), kmin=kmin, triangles=True)
    o = O.graph_stats(rp, col, kmin=kmin, triangles=True)
    assert g["ascending_rows"] == 1
    assert g["hist"] == list(o["hist"]) and g["max_degree"] == o["max_degree"]
    assert g["tail_count"] == o["tail_count"] and g["triads"] == o["triads"]
    assert g["triangles"] == o["triangles"]
    for f in ("gamma_mle", "assortativity", "transitivity", "avg_local_clustering"):
        assert _close(g[f], o[f]), (f, g[f], o[f])
    return g


def _csr(n, pairs):
    rows = [set() for _ in range(n)]
    for a, b in pairs:
        rows[a].add(b)
        rows[b].add(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in sorted(r)], dtype=np.int32)
    return rp, col


def test_named_graphs():
    n = 9
    g = _compare(*_csr(n, itertools.combinations(range(n), 2)))
    assert g["triangles"] == math.comb(n, 3) and g["transitivity"] == 1.0
    g = _compare(*_csr(n, [(0, v) for v in range(1, n)]), kmin=1.0)
    assert g["triangles"] == 0 and g["assortativity"] == -1.0
    m = 12
    pairs = [(0, v) for v in range(1, m + 1)] + [(v, v % m + 1) for v in range(1, m + 1)]
    assert _compare(*_csr(m + 1, pairs))["triangles"] == m
    assert _compare(*_csr(4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]))["triangles"] == 2


def test_brute_force_graph():
    n, k_bar, g = 3000, 10.0, 2.5
    a_, R = O.solve_R(n, k_bar, g)
    r, t, _ = O.sample(4, a_, R, n)
    rp, col = O.csr(r, t, R)[:2]
    s = _compare(rp, col, kmin=10.0)
    _say("n=3000:", {k: s[k] for k in ("triangles", "transitivity", "avg_local_clustering", "gamma_mle")})


def test_generated_graph_and_run_to_run_bits():
    import torch
    gr = P.rhg_generate(20_000, 10.0, 2.2, 5, canonical_rows=True)
    rp, col = gr.row_ptr.cpu().numpy(), gr.col_idx.cpu().numpy()
    s = _compare(rp, col, kmin=10.0)
    _say("n=2e4 gamma=2.2:", {k: s[k] for k in ("triangles", "transitivity", "avg_local_clustering", "gamma_mle",
                                                 "assortativity", "max_degree")})
    s2 = P.rhg_graph_stats(gr.row_ptr, gr.col_idx, kmin=10.0)
    assert s2 == s
    # search-order rows: everything but the triangles
    raw = P.rhg_generate(20_000, 10.0, 2.2, 5)
    s3 = P.rhg_graph_stats(raw.row_ptr, raw.col_idx, kmin=10.0, triangles=False)
    assert s3["ascending_rows"] == 0 and s3["triangles"] == -1
    for f in ("hist", "max_degree", "tail_count", "triads"):
        assert s3[f] == s[f]
    with pytest.raises(P.RhgError):
        P.rhg_graph_stats(raw.row_ptr, raw.col_idx, kmin=10.0, triangles=True)
    torch.cuda.synchronize()


def test_degenerate_graphs():
    import torch
    s = P.rhg_graph_stats(torch.zeros(1, dtype=torch.int64, device="cuda"),
                          torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert s["n"] == 0 and s["triangles"] == 0 and sum(s["hist"]) == 0
    s = P.rhg_graph_stats(torch.zeros(6, dtype=torch.int64, device="cuda"),
                          torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert s["hist"][0] == 5 and s["triangles"] == 0 and math.isnan(s["transitivity"])
    _compare(*_csr(2, [(0, 1)]), kmin=1.0)
