"""Helpers shared by the GPU tests: run the library through its C ABI and
compare CSR graphs with the oracle's."""
import numpy as np



def run_search(P, params, r_np, t_np, tuning=None, validate=True):
    """build_index + count + emit on device for given host points; returns
    (row_ptr, col, stats) as numpy arrays."""
    import torch
    n = int(params.n)
    r = torch.from_numpy(np.ascontiguousarray(r_np, dtype=np.float64)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(t_np, dtype=np.float64)).cuda()
    idx = P.rhg_build_index(params, r, t, tuning=tuning, validate=validate)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    P.rhg_count_edges(idx, row_ptr)
    nnz = int(row_ptr[-1].item())
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    P.rhg_emit_edges(idx, row_ptr, col[:nnz] if nnz else col[:0])
    stats = P.rhg_index_stats(idx)
    torch.cuda.synchronize()
    out = row_ptr.cpu().numpy(), col[:nnz].cpu().numpy(), stats
    idx.free()
    return out


def canonical(row_ptr, col):
    """Rows sorted ascending (the oracle's order)."""
    n = row_ptr.shape[0] - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    order = np.lexsort((col, src))
    return col[order]


def check_simple_symmetric(row_ptr, col):
    n = row_ptr.shape[0] - 1
    assert row_ptr[0] == 0 and np.all(np.diff(row_ptr) >= 0)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    assert not np.any(src == col), "self-loop"
    fwd = np.sort(src * n + col)
    assert np.all(np.diff(fwd) > 0), "duplicate edge"
    bwd = np.sort(col.astype(np.int64) * n + src)
    assert np.array_equal(fwd, bwd), "not symmetric"


def ulp_diff(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    return np.abs(ia - ib)


def pipeline_compare(g, r_o, t_o, R, orp, ocol):
    """GPU pipeline vs oracle pipeline: angles and radii bit for bit, then
    the edge sets; returns the number of edges in one set only (pairs within
    an ulp-scale change of the threshold are reported, not excused)."""
    tg = g.theta.cpu().numpy()
    rg = g.r.cpu().numpy()
    assert np.array_equal(tg, t_o)
    assert np.array_equal(rg, r_o), "radii differ: max %d ulp" % ulp_diff(rg, r_o).max()
    rp = g.row_ptr.cpu().numpy()
    col = g.col_idx.cpu().numpy()
    check_simple_symmetric(rp, col)
    n = rp.shape[0] - 1
    a = set((np.repeat(np.arange(n), np.diff(rp)) * n + col).tolist())
    b = set((np.repeat(np.arange(n), np.diff(orp)) * n + ocol).tolist())
    return len(a ^ b)


def oracle_check(O, g, d, full_limit=20_000, rows=24):
    """One generated graph g (theta, r, row_ptr, col_idx on the device) of
    request d against the oracle: the points bit for bit, then the whole edge
    set for n <= full_limit, else `rows` rows (stratified by radius, plus the
    largest degrees) each tested against all n points.  Returns what it
    checked."""
    n, k, gamma, seed = d["n"], d["avg_degree"], d["gamma"], d["seed"]
    a, R = O.solve_R(n, k, gamma)
    assert (a, R) == (g.params.alpha, g.params.R)
    if n <= full_limit:
        _, _, r_o, t_o, orp, ocol, st = O.generate(n, k, gamma, seed)
        assert st["ties"] == 0
        assert pipeline_compare(g, r_o, t_o, R, orp, ocol) == 0
        return "full"
    r_o, t_o, hard = O.sample(seed, a, R, n)
    assert hard == 0
    assert np.array_equal(g.theta.cpu().numpy(), t_o)
    assert np.array_equal(g.r.cpu().numpy(), r_o)
    rp = g.row_ptr.cpu().numpy()
    col = g.col_idx.cpu().numpy()
    deg = np.diff(rp)
    order = np.argsort(r_o, kind="stable")
    which = np.unique(np.concatenate([order[np.linspace(0, n - 1, rows - rows // 3).astype(np.int64)],
                                      np.argsort(deg)[-(rows // 3):]]).astype(np.int64))
    ptr, ocol, _, nt = O.rows(r_o, t_o, R, which)
    assert nt == 0
    for a_, i in enumerate(which):
        assert np.array_equal(np.sort(col[rp[i]:rp[i + 1]]), ocol[ptr[a_]:ptr[a_ + 1]]), (d, i)
    return "rows"
