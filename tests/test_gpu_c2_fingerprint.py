"""C2 (n = 1e6, average degree 10, gamma 2.7, seed 2) as a whole graph: the
GPU's degree array and order-independent edge fingerprint against the
oracle's brute force over all 5e11 pairs, which a script that calls only the
oracle stored under tests/golden."""
import sys

import numpy as np
import pytest

import paper_1501_03545_amd as P
from gpu_util import check_simple_symmetric

pytestmark = pytest.mark.gpu

C2 = (1_000_000, 10.0, 2.7)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c2_whole_graph_equals_the_oracle_fingerprint():
    """n = 1e6, average degree 10, gamma 2.7, seed 2: the degree array and
    the order-independent edge fingerprint of the whole graph equal the
    oracle's brute force over all 5e11 pairs (stored under tests/golden by a
    script that calls only the oracle)."""
    import json
    import os
    from fingerprint import csr_fingerprint, degree_sha256
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2_fingerprint.json")) as f:
        gold = json.load(f)
    n, k, g_ = C2
    assert (gold["n"], gold["avg_degree"], gold["gamma"], gold["seed"]) == (n, k, g_, 2)
    assert gold["ties"] == 0
    g = P.rhg_generate(n, k, g_, 2)
    assert g.params.R == gold["R"] and float.fromhex(gold["R_hex"]) == g.params.R
    rp = g.row_ptr.cpu().numpy()
    col = g.col_idx.cpu().numpy()
    check_simple_symmetric(rp, col)
    deg = np.diff(rp).astype(np.int32)
    _say("C2 edges", col.size // 2, "oracle", gold["undirected_edges"])
    assert col.size // 2 == gold["undirected_edges"]
    assert degree_sha256(deg) == gold["degree_sha256"]
    fs, fx = csr_fingerprint(rp, col)
    assert ("%016x" % fs, "%016x" % fx) == (gold["fingerprint_sum"], gold["fingerprint_xor"])
