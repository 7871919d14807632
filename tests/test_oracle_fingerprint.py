"""Pins of the oracle's whole-graph summary (degrees and the order-independent
edge fingerprint) and of its blocked row check, against the oracle's full
CSR and against a numpy fingerprint written apart from it."""
import numpy as np
import pytest

import oracle as O
from fingerprint import csr_fingerprint, mix64


@pytest.fixture(scope="module")
def c1():
    a, R, r, t, rp, col, st = O.generate(10_000, 6.0, 3.0, 1)
    return R, r, t, rp, col


def test_mix64_matches_the_numpy_finaliser():
    for z in [0, 1, 2, 0xFFFFFFFF, 1 << 32, (1 << 64) - 1, 0x0123456789ABCDEF]:
        assert int(mix64(z)) == O.mix64(z)
    # SplitMix64's first output for seed 0 is the finaliser of the golden gamma
    assert O.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_pair_scan_equals_the_csr(c1):
    R, r, t, rp, col = c1
    deg, fs, fx, quad, ties = O.pair_scan(r, t, R)
    assert ties == 0
    assert np.array_equal(deg, np.diff(rp))
    assert (fs, fx) == csr_fingerprint(rp, col)


def test_fingerprint_sees_one_missing_or_moved_edge(c1):
    R, r, t, rp, col = c1
    base = csr_fingerprint(rp, col)
    n = rp.size - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    k = int(np.flatnonzero(col > src)[17])
    i, j = int(src[k]), int(col[k])
    # drop the edge {i, j} from both rows
    keep = ~(((src == i) & (col == j)) | ((src == j) & (col == i)))
    rp2 = np.zeros_like(rp)
    np.cumsum(np.bincount(src[keep], minlength=n), out=rp2[1:])
    assert csr_fingerprint(rp2, col[keep]) != base
    # move it to {i, j + 1} (same edge count, same degree sum)
    col3 = col.copy()
    col3[k] = j + 1 if j + 1 != i else j + 2
    assert csr_fingerprint(rp, col3) != base


def test_row_blocks_equal_the_csr_rows(c1):
    R, r, t, rp, col = c1
    # more rows than one block, with repeats and the extremes of the radius
    which = np.concatenate([np.argsort(r)[:40], np.arange(0, 10_000, 397), [5, 5]]).astype(np.int64)
    ptr, oc, _, ties = O.rows(r, t, R, which)
    assert ties == 0
    for a, i in enumerate(which):
        assert np.array_equal(oc[ptr[a]:ptr[a + 1]], col[rp[i]:rp[i + 1]]), i
