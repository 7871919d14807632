"""Pins of the oracle's long-range augmentation (RHG-LR): the candidate
pairs are the published Philox words mapped to vertices exactly as stated,
they are uniform, and the augmentation adds exactly the first k admissible
candidates (no self-loop, no existing edge, no repeat) to a simple symmetric
graph, saturating gracefully when few pairs are left."""
import math

import numpy as np
import pytest

import oracle as O


def setup_module(_):
    O.build(force=False)


def _words(seed, j):
    x = O.philox4x32_10([j & 0xFFFFFFFF, j >> 32, 1, 0], [seed & 0xFFFFFFFF, seed >> 32])
    return (int(x[1]) << 32) | int(x[0]), (int(x[3]) << 32) | int(x[2])


def test_candidates_are_the_philox_words_mapped_by_integer_arithmetic():
    seed, n = 0x1234_5678_9ABC, 1_000_003
    a, b = O.lr_candidates(seed, 7, 50, n)
    for c in range(50):
        w0, w1 = _words(seed, 7 + c)
        u, v = (w0 * n) >> 64, (w1 * n) >> 64  # exact big-integer products
        assert (a[c], b[c]) == (min(u, v), max(u, v))
    # the third counter word keeps them apart from the points' draws
    pt = O.philox4x32_10([7, 0, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
    assert (int(pt[1]) << 32 | int(pt[0])) != _words(seed, 7)[0]


def test_candidate_vertices_are_uniform():
    n, count = 40, 200_000
    a, b = O.lr_candidates(9, 0, count, n)
    hits = np.bincount(np.concatenate([a, b]), minlength=n)
    expect = 2 * count / n
    chi2 = float(((hits - expect) ** 2 / expect).sum())
    assert chi2 < 39 + 5 * math.sqrt(2 * 39)  # 39 degrees of freedom, > 5 sigma off
    # a self-loop has probability 1/n
    assert abs(float(np.mean(a == b)) - 1 / n) < 5 * math.sqrt(1 / n / count)


def _csr_from_pairs(n, pairs):
    rows = [[] for _ in range(n)]
    for a, b in pairs:
        rows[a].append(b)
        rows[b].append(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in sorted(r)], dtype=np.int32)
    return rp, col


def test_augmentation_adds_exactly_the_first_k_admissible_candidates():
    n, k_bar, g = 3000, 10.0, 2.5
    a_, R = O.solve_R(n, k_bar, g)
    r, t, _ = O.sample(4, a_, R, n)
    rp, col = O.csr(r, t, R)[:2]
    m = int(rp[-1]) // 2
    k = math.ceil(0.005 * m)
    seed = 77
    orp, ocol, added = O.lr_augment(n, rp, col, k, seed)
    assert added == k
    # a second, vectorised reading of the definition over the drawn candidates
    ca, cb = O.lr_candidates(seed, 0, O.lr_draw_limit(k), n)
    keys = ca * n + cb
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    existing = np.isin(keys, src * n + col.astype(np.int64))
    _, first = np.unique(keys, return_index=True)
    is_first = np.zeros(keys.size, dtype=bool)
    is_first[first] = True
    ok = (ca != cb) & ~existing & is_first
    chosen = np.flatnonzero(ok)[:k]
    want = set(zip(ca[chosen].tolist(), cb[chosen].tolist()))
    assert set(O.lr_added_pairs(n, rp, col, k, seed)) == want
    # the augmented graph: simple, symmetric, old rows kept as prefixes
    deg_old, deg_new = np.diff(rp), np.diff(orp)
    assert int(orp[-1]) == int(rp[-1]) + 2 * k
    s2 = np.repeat(np.arange(n, dtype=np.int64), deg_new)
    assert not np.any(s2 == ocol)
    fwd = np.sort(s2 * n + ocol)
    assert np.all(np.diff(fwd) > 0)
    assert np.array_equal(fwd, np.sort(ocol.astype(np.int64) * n + s2))
    for v in range(0, n, 97):
        assert np.array_equal(ocol[orp[v]:orp[v] + deg_old[v]], col[rp[v]:rp[v + 1]])
    # the added edges are spread over the vertices, not over the graph's edges
    extra = deg_new - deg_old
    assert extra.sum() == 2 * k and extra.max() <= 6


def test_saturation_and_degenerate_graphs():
    # complete graph: nothing can be added
    n = 25
    rp, col = _csr_from_pairs(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    assert O.lr_augment(n, rp, col, 10, 3)[2] == 0
    # all but five pairs present: exactly those five are added
    missing = [(0, 1), (2, 7), (3, 19), (10, 11), (4, 24)]
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in missing]
    rp, col = _csr_from_pairs(n, pairs)
    assert set(O.lr_added_pairs(n, rp, col, 10, 5)) == set(missing)
    # empty graph on one vertex: only self-loops can be drawn
    assert O.lr_augment(1, np.zeros(2, dtype=np.int64), np.zeros(0, dtype=np.int32), 3, 1)[2] == 0
    # k = 0
    orp, ocol, added = O.lr_augment(n, rp, col, 0, 5)
    assert added == 0 and np.array_equal(orp, rp) and np.array_equal(ocol, col)
