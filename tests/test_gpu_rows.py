"""Canonical rows on the GPU: rhg_sort_rows sorts every length class (ranked
short rows, wavefront rows, workgroup rows, tiled long rows with merge
levels in global memory) exactly as a host sort does, and the canonical emit
gives the oracle's ascending rows byte for byte, the same for every tuning."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from gpu_util import canonical

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _host_sorted(row_ptr, col):
    n = row_ptr.shape[0] - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    return col[np.lexsort((col, src))]


def _sort_on_device(lengths, rng, lo=-2**31, hi=2**31, nnz_extra=0):
    import torch
    lengths = np.asarray(lengths, dtype=np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    nnz = int(row_ptr[-1])
    col = rng.integers(lo, hi, size=nnz, dtype=np.int64).astype(np.int32)
    d_rp = torch.from_numpy(row_ptr).cuda()
    d_col = torch.from_numpy(col.copy()).cuda()
    P.rhg_sort_rows(d_rp, d_col, nnz=nnz + nnz_extra)
    torch.cuda.synchronize()
    return row_ptr, col, d_col.cpu().numpy()


def test_every_length_class_sorts_like_the_host():
    rng = np.random.default_rng(7)
    # class edges: 1 | 2..64 ranked | 65..512 wavefront | 513..8192 workgroup |
    # longer: tiles of 8192 and merge levels (up to 2^18 here)
    edges = [0, 1, 2, 3, 63, 64, 65, 66, 127, 128, 511, 512, 513, 1000, 4096, 8191, 8192, 8193,
             12000, 16384, 16385, 24577, 65536, 100003, 262145]
    small = rng.integers(0, 40, size=3000)
    lengths = np.concatenate([small[:1500], edges, small[1500:], edges[::-1]])
    _say("rows", lengths.size, "entries", int(lengths.sum()))
    row_ptr, col, got = _sort_on_device(lengths, rng)
    assert np.array_equal(got, _host_sorted(row_ptr, col))


def test_duplicates_narrow_ranges_and_extreme_values():
    rng = np.random.default_rng(8)
    lengths = [5, 64, 200, 5000, 20000, 0, 1, 70000]
    # few distinct values: many ties in every class
    row_ptr, col, got = _sort_on_device(lengths, rng, lo=-3, hi=4)
    assert np.array_equal(got, _host_sorted(row_ptr, col))
    # the extremes of int32
    row_ptr, col, got = _sort_on_device(lengths, rng, lo=-2**31, hi=-2**31 + 2)
    assert np.array_equal(got, _host_sorted(row_ptr, col))
    row_ptr, col, got = _sort_on_device(lengths, rng, lo=2**31 - 2, hi=2**31)
    assert np.array_equal(got, _host_sorted(row_ptr, col))


def test_sorted_and_reversed_rows_and_a_loose_nnz_bound():
    import torch
    lengths = np.array([3, 70, 600, 9000, 40000, 33], dtype=np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    parts = []
    for k, L in enumerate(lengths):
        v = np.arange(L, dtype=np.int32) * 3 - 7
        parts.append(v if k % 2 else v[::-1])
    col = np.concatenate(parts)
    d_rp = torch.from_numpy(row_ptr).cuda()
    d_col = torch.from_numpy(col.copy()).cuda()
    # an nnz bound far above the real count only adds merge levels that exit
    P.rhg_sort_rows(d_rp, d_col, nnz=int(row_ptr[-1]) * 1000)
    torch.cuda.synchronize()
    assert np.array_equal(d_col.cpu().numpy(), _host_sorted(row_ptr, col))


def test_empty_inputs_and_errors():
    import torch
    rp = torch.zeros(1, dtype=torch.int64, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    P.rhg_sort_rows(rp, col)  # n = 0
    rp = torch.zeros(11, dtype=torch.int64, device="cuda")
    P.rhg_sort_rows(rp, col)  # ten empty rows, nnz = 0
    rp = torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda")
    col = torch.tensor([5, 1, 9, -4], dtype=torch.int32, device="cuda")
    with pytest.raises(P.RhgError):
        P.rhg_sort_rows(rp, col, workspace=torch.empty(8, dtype=torch.uint8, device="cuda"))
    P.rhg_sort_rows(rp, col)
    torch.cuda.synchronize()
    assert col.cpu().tolist() == [1, 5, -4, 9]


def test_canonical_emit_is_the_oracle_csr_c1():
    n, k, g_ = 10_000, 6.0, 3.0
    g = P.rhg_generate(n, k, g_, 1, canonical_rows=True)
    a, R, r_o, t_o, orp, ocol, st = O.generate(n, k, g_, 1)
    assert st["ties"] == 0
    assert np.array_equal(g.row_ptr.cpu().numpy(), orp)
    assert np.array_equal(g.col_idx.cpu().numpy(), ocol)


def test_canonical_rows_are_the_same_bytes_for_every_tuning():
    import torch
    n, k, g_, seed = 200_000, 64.0, 2.1, 11
    outs = []
    for tun in (None, {"band_width": 1.0, "cell_target": 4, "heavy_points": 2048},
                {"band_width": 3.0, "sweep_max": -1}):
        g = P.rhg_generate(n, k, g_, seed, tuning=tun, canonical_rows=True)
        outs.append((g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy()))
        raw = P.rhg_generate(n, k, g_, seed, tuning=tun)
        rp, col = raw.row_ptr.cpu().numpy(), raw.col_idx.cpu().numpy()
        assert np.array_equal(outs[-1][1], canonical(rp, col))
        del g, raw
        torch.cuda.empty_cache()
    deg = np.diff(outs[0][0])
    _say("max degree", int(deg.max()), "rows above 8192:", int((deg > 8192).sum()))
    assert deg.max() > 2 * 8192, "the workload should exercise the merge levels"
    for rp, col in outs[1:]:
        assert np.array_equal(rp, outs[0][0]) and np.array_equal(col, outs[0][1])


def test_canonical_rows_at_n_1e7_are_ascending_and_hold_the_same_entries():
    import torch
    n, k, g_, seed = 10_000_000, 16.0, 2.5, 5
    raw = P.rhg_generate(n, k, g_, seed)
    can = P.rhg_generate(n, k, g_, seed, canonical_rows=True)
    assert torch.equal(raw.row_ptr, can.row_ptr)
    rp = can.row_ptr
    deg = rp[1:] - rp[:-1]
    nnz = int(rp[-1].item())
    src = torch.repeat_interleave(torch.arange(n, device="cuda"), deg)
    c = can.col_idx.long()
    inner = src[1:] == src[:-1]
    assert bool(torch.all(c[1:][inner] > c[:-1][inner])), "a row is not strictly ascending"
    # the same multiset per row: per-row sums of two mixes of the entries
    for f in (lambda x: x, lambda x: (x * 0x9E3779B1) % 1000003):
        a = torch.zeros(n, dtype=torch.int64, device="cuda").index_add_(0, src, f(raw.col_idx.long()))
        b = torch.zeros(n, dtype=torch.int64, device="cuda").index_add_(0, src, f(c))
        assert torch.equal(a, b)
    _say("n=1e7 canonical rows ok, nnz", nnz, "max degree", int(deg.max().item()))
