"""Long-range augmentation on the GPU (rhg_long_range through the C ABI)
against the oracle's sequential definition: the same extra edges in the same
places, byte for byte, on brute-force graphs, on generated graphs in both row
orders, on a graph whose shorter rows are long (the workgroup membership
check), and in the saturated and degenerate cases."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _run(rp, col, k, seed):
    import torch
    d_rp = torch.from_numpy(np.asarray(rp, dtype=np.int64)).cuda()
    d_col = torch.from_numpy(np.asarray(col, dtype=np.int32)).cuda()
    n = rp.shape[0] - 1
    orp, ocol, added = P.rhg_long_range(d_rp, d_col, k, seed, nnz=int(rp[-1]))
    torch.cuda.synchronize()
    a = int(added.item())
    return orp.cpu().numpy(), ocol[:int(rp[-1]) + 2 * a].cpu().numpy(), a


def _check(rp, col, k, seed):
    n = rp.shape[0] - 1
    g_rp, g_col, g_add = _run(rp, col, k, seed)
    o_rp, o_col, o_add = O.lr_augment(n, rp, col, k, seed)
    assert g_add == o_add
    assert np.array_equal(g_rp, o_rp)
    assert np.array_equal(g_col, o_col)
    return g_add


def _csr_from_pairs(n, pairs):
    rows = [[] for _ in range(n)]
    for a, b in pairs:
        rows[a].append(b)
        rows[b].append(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in r], dtype=np.int32)
    return rp, col


def test_oracle_graph_matches_the_definition():
    n, k_bar, g = 3000, 10.0, 2.5
    a_, R = O.solve_R(n, k_bar, g)
    r, t, _ = O.sample(4, a_, R, n)
    rp, col = O.csr(r, t, R)[:2]
    k = P.long_range_count(int(rp[-1]) // 2)
    for seed in (77, 2**40 + 5):
        assert _check(rp, col, k, seed) == k


@pytest.mark.parametrize("canonical", [False, True])
def test_generated_graph_in_either_row_order(canonical):
    n, k_bar, g = 200_000, 10.0, 2.2
    gr = P.rhg_generate(n, k_bar, g, 9, canonical_rows=canonical)
    rp, col = gr.row_ptr.cpu().numpy(), gr.col_idx.cpu().numpy()
    k = P.long_range_count(int(rp[-1]) // 2)
    _say("n", n, "m", int(rp[-1]) // 2, "k", k)
    assert _check(rp, col, k, 31) == k


def test_long_shorter_rows_use_the_workgroup_check():
    # a clique on 600 vertices (rows of 599 > 256 entries) plus a sparse rest:
    # about a third of the candidates fall inside the clique and are rejected
    # by the workgroup scan
    rng = np.random.default_rng(5)
    n = 1000
    pairs = {(a, b) for a in range(600) for b in range(a + 1, 600)}
    while len(pairs) < 600 * 599 // 2 + 1500:
        a, b = sorted(rng.integers(0, n, 2).tolist())
        if a != b and b >= 600:
            pairs.add((a, b))
    rp, col = _csr_from_pairs(n, sorted(pairs, key=lambda p: rng.random()))
    added = _check(rp, col, 2000, 3)
    _say("clique graph: added", added)
    assert added == 2000


def test_saturated_tiny_and_empty_graphs():
    n = 25
    rp, col = _csr_from_pairs(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    assert _check(rp, col, 10, 3) == 0
    missing = [(0, 1), (2, 7), (3, 19), (10, 11), (4, 24)]
    rp, col = _csr_from_pairs(n, [(a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in missing])
    assert _check(rp, col, 10, 5) == 5
    assert _check(rp, col, 0, 5) == 0
    # one vertex, no edges: only self-loops can be drawn
    assert _check(np.zeros(2, dtype=np.int64), np.zeros(0, dtype=np.int32), 4, 1) == 0
    # no edges at all on 50 vertices
    assert _check(np.zeros(51, dtype=np.int64), np.zeros(0, dtype=np.int32), 30, 8) == 30


def test_errors_are_reported():
    import torch
    rp = torch.zeros(11, dtype=torch.int64, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    with pytest.raises(P.RhgError):
        P.rhg_long_range(rp, col, 5, 1, out=(torch.empty(11, dtype=torch.int64, device="cuda"),
                                             torch.empty(3, dtype=torch.int32, device="cuda")))
    with pytest.raises(P.RhgError):
        P.rhg_long_range(rp, col, 5, 1, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
