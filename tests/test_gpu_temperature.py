"""GPU parity of the temperature model: the HIP path through the C ABI
against the oracle's brute force (every pair with its coin), entry for entry
on canonical rows.  Covers the FP32 screen and the exact stages, the heavy
(chunked) and light (lane per query) work, several tunings, the whole
pipeline, sampled rows of the n = 1e6 graph, and the error paths."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from gpu_util import canonical, check_simple_symmetric

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _run_temp(params, r_np, t_np, T, tuning=None, canonical_rows=False, twice=False):
    import torch
    n = int(params.n)
    r = torch.from_numpy(np.ascontiguousarray(r_np, dtype=np.float64)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(t_np, dtype=np.float64)).cuda()
    idx = P.rhg_build_index(params, r, t, tuning=tuning, validate=True)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    P.rhg_temp_count_edges(idx, T, row_ptr)
    if twice:
        first = row_ptr.clone()
        P.rhg_temp_count_edges(idx, T, row_ptr)
        assert torch.equal(first, row_ptr)
    nnz = int(row_ptr[-1].item())
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    P.rhg_temp_emit_edges(idx, T, row_ptr, col[:nnz], canonical_rows=canonical_rows)
    stats = P.rhg_index_stats(idx)
    torch.cuda.synchronize()
    out = row_ptr.cpu().numpy(), col[:nnz].cpu().numpy(), stats
    idx.free()
    return out


def _oracle_points(n, k, g, seed):
    a, R = O.solve_R(n, k, g)
    r, t, hard = O.sample(seed, a, R, n)
    assert hard == 0
    return P.rhg_plan_radius(n, a, R, seed), a, R, r, t


# (n, average degree, gamma, T, seed): several tiles and a ragged tail,
# heavy-tailed and light-tailed radii, cold and warm temperatures
CASES = [(2_000, 6.0, 3.0, 0.05, 1), (5_000, 10.0, 2.5, 0.3, 2), (20_000, 8.0, 2.2, 0.5, 3),
         (12_001, 6.0, 3.0, 0.9, 4), (3_000, 20.0, 2.7, 0.1, 5), (10_000, 6.0, 3.0, 0.2, 1),
         (777, 40.0, 2.1, 0.7, 6)]


@pytest.mark.parametrize("case", CASES)
def test_temperature_edge_set_equals_oracle(case):
    n, k, g, T, seed = case
    _say("temperature parity", case)
    p, a, R, r, t = _oracle_points(n, k, g, seed)
    orp, ocol, _, ties = O.temp_csr(r, t, R, T, seed)
    assert ties == 0
    rp, col, st = _run_temp(p, r, t, T, twice=True)
    _say("edges", int(rp[-1]) // 2, "oracle", int(orp[-1]) // 2, "stats", st)
    assert st["ties"] == 0
    check_simple_symmetric(rp, col)
    assert np.array_equal(rp, orp)
    assert np.array_equal(canonical(rp, col), ocol)


TUNINGS = [{"fp64_only": 1}, {"exact_inline": 1}, {"defer_cap": 1}, {"heavy_points": 64},
           {"heavy_points": 1 << 16}, {"band_width": 1.0}, {"band_width": 3.0, "cell_target": 4},
           {"inner_radius": 1e-9}]


def test_temperature_tunings_give_the_same_edges():
    n, k, g, T, seed = 15_000, 12.0, 2.4, 0.4, 9
    p, a, R, r, t = _oracle_points(n, k, g, seed)
    orp, ocol, _, ties = O.temp_csr(r, t, R, T, seed)
    assert ties == 0
    for tu in TUNINGS:
        _say("tuning", tu)
        rp, col, st = _run_temp(p, r, t, T, tuning=tu)
        assert np.array_equal(rp, orp), tu
        assert np.array_equal(canonical(rp, col), ocol), tu
        if tu.get("fp64_only"):
            assert st["fp32_undecided"] == 0
    # canonical rows straight from the library
    rp, col, _ = _run_temp(p, r, t, T, canonical_rows=True)
    assert np.array_equal(col, ocol)


def test_temperature_staged_rows_are_the_search_rows():
    """Staged (the count pass writes the light rows into their slots, the
    emit pass copies them) and unstaged runs of the same tuning give the
    same bytes in search order: slots that fit, slots too small for most
    rows (their wavefronts searched again), an overflowed undecided-pair
    list, hubs among the light queries, and both exact-only modes."""
    n, k, g, T, seed = 15_000, 12.0, 2.4, 0.4, 9
    p, a, R, r, t = _oracle_points(n, k, g, seed)
    orp, ocol, _, ties = O.temp_csr(r, t, R, T, seed)
    assert ties == 0
    for tu in ({}, {"stage_pct": 1}, {"defer_cap": 1}, {"heavy_points": 64}, {"exact_inline": 1},
               {"fp64_only": 1}):
        _say("staged", tu)
        rp0, col0, _ = _run_temp(p, r, t, T, tuning=dict(tu, stage=-1))
        rp, col, st = _run_temp(p, r, t, T, tuning=dict(tu, stage=1), twice=True)
        _say("stats", st)
        assert st["staged_waves"] > 0
        if tu.get("stage_pct"):
            assert st["stage_overflows"] > 0
        assert np.array_equal(rp, orp), tu
        assert np.array_equal(rp, rp0) and np.array_equal(col, col0), tu
        assert np.array_equal(canonical(rp, col), ocol), tu


def test_temperature_cold_graph_in_every_exact_mode():
    # a cold graph: the coins' boundaries D(u) stay near R, where many pairs lie
    n, k, g, T, seed = 20_000, 10.0, 2.3, 0.01, 11
    p, a, R, r, t = _oracle_points(n, k, g, seed)
    orp, ocol, _, ties = O.temp_csr(r, t, R, T, seed)
    assert ties == 0
    for tu in (None, {"exact_inline": 1}, {"defer_cap": 2}, {"stage": 1}, {"stage": 1, "defer_cap": 2}):
        rp, col, st = _run_temp(p, r, t, T, tuning=tu)
        _say("stats", tu, st)
        assert st["ties"] == 0
        assert 0 < st["temp_coins"] <= st["temp_candidates"]
        assert np.array_equal(rp, orp)
        assert np.array_equal(canonical(rp, col), ocol)


def _near_boundary_points(n, k, g, T, seed, m, rng):
    """The sampler's points, then m of them moved so that their pair with
    point 0 lies at a relative distance 2^-e (e = 12 .. 44) from the pair's
    coin boundary D(u) = R + 2T ln((1 - u)/u): the FP32 stage cannot decide
    these pairs, and the closest ones reach double-double."""
    import mpmath as mp
    mp.mp.dps = 50
    a, R = O.solve_R(n, k, g)
    r, t, _ = O.sample(seed, a, R, n)
    r, t = r.copy(), t.copy()
    r[0], t[0] = 0.8 * R, 1.0
    placed = 0
    for j in range(1, n):
        if placed == m:
            break
        cu = mp.mpf(O.temp_coin(seed, 0, j)) / 2**53
        D = mp.mpf(R) + 2 * mp.mpf(T) * mp.log((1 - cu) / cu)
        rj = float(R * (0.55 + 0.45 * rng.random()))
        e = int(rng.integers(12, 45))
        target = D * (1 + (1 if rng.random() < 0.5 else -1) * mp.mpf(2) ** (-e))
        if not (abs(r[0] - rj) < target < r[0] + rj):
            continue
        c = (mp.cosh(target) - mp.cosh(mp.mpf(r[0]) - rj)) / (2 * mp.sinh(r[0]) * mp.sinh(rj))
        tj = float(t[0] + 2 * mp.asin(mp.sqrt(c)) * (1 if rng.random() < 0.5 else -1))
        if not (0.0 <= tj < 6.283185307179586):
            continue
        r[j], t[j] = rj, tj
        placed += 1
    assert placed == m
    return P.rhg_plan_radius(n, a, R, seed), R, r, t


@pytest.mark.parametrize("T", [0.05, 0.5])
def test_temperature_pairs_at_the_coin_boundary(T):
    rng = np.random.default_rng(int(T * 100))
    p, R, r, t = _near_boundary_points(4_000, 8.0, 2.5, T, 31, 300, rng)
    orp, ocol, quad, ties = O.temp_csr(r, t, R, T, 31)
    assert ties == 0 and quad > 0
    for tu in (None, {"fp64_only": 1}, {"exact_inline": 1}, {"stage": 1}):
        rp, col, st = _run_temp(p, r, t, T, tuning=tu)
        _say("near boundary", T, tu, st)
        assert st["ties"] == 0
        if tu is None or tu.get("stage"):
            assert st["fp32_undecided"] > 0 and st["dd_fallbacks"] > 0
        assert np.array_equal(rp, orp)
        assert np.array_equal(canonical(rp, col), ocol)


def test_temperature_whole_pipeline_against_oracle():
    n, k, g, T, seed = 9_000, 8.0, 2.6, 0.25, 21
    G = P.rhg_temp_generate(n, k, g, T, seed, canonical_rows=True)
    a, R = O.solve_R(n, k, g)
    assert (G.params.alpha, G.params.R) == (a, R)
    r, t, _ = O.sample(seed, a, R, n)
    assert np.array_equal(G.r.cpu().numpy(), r) and np.array_equal(G.theta.cpu().numpy(), t)
    orp, ocol, _, ties = O.temp_csr(r, t, R, T, seed)
    assert ties == 0
    assert np.array_equal(G.row_ptr.cpu().numpy(), orp)
    assert np.array_equal(G.col_idx.cpu().numpy(), ocol)


def test_temperature_n1e6_sampled_rows_against_oracle():
    """The n = 1e6, average degree 10, gamma = 2.7 graph at T = 0.1: rows
    stratified by radius plus the largest degrees, each against all n
    points with their coins."""
    n, k, g, T, seed = 1_000_000, 10.0, 2.7, 0.1, 2
    _say("temperature n=1e6")
    G = P.rhg_temp_generate(n, k, g, T, seed)
    a, R = O.solve_R(n, k, g)
    r, t, _ = O.sample(seed, a, R, n)
    assert np.array_equal(G.r.cpu().numpy(), r)
    rp = G.row_ptr.cpu().numpy()
    col = G.col_idx.cpu().numpy()
    deg = np.diff(rp)
    _say("edges", int(rp[-1]) // 2, "mean degree", float(deg.mean()))
    order = np.argsort(r, kind="stable")
    which = np.unique(np.concatenate([order[np.linspace(0, n - 1, 160).astype(np.int64)],
                                      np.argsort(deg)[-40:]]).astype(np.int64))
    ptr, ocol, _, nt = O.temp_rows(r, t, R, T, seed, which)
    assert nt == 0
    for j, i in enumerate(which):
        assert np.array_equal(np.sort(col[rp[i]:rp[i + 1]]), ocol[ptr[j]:ptr[j + 1]]), i


def test_temperature_degenerate_sizes():
    import torch
    for n in (0, 1, 2, 3, 65):
        a, R = 0.75, 5.0
        p = P.rhg_plan_radius(n, a, R, 3)
        r, t, _ = O.sample(3, a, R, n) if n else (np.zeros(0), np.zeros(0), 0)
        orp, ocol, _, _ = O.temp_csr(np.asarray(r), np.asarray(t), R, 0.5, 3)
        for tu in (None, {"stage": 1}, {"stage": 1, "stage_pct": 1}):
            rp, col, st = _run_temp(p, r, t, 0.5, tuning=tu)
            assert np.array_equal(rp, orp) and np.array_equal(canonical(rp, col), ocol), (n, tu)
    torch.cuda.synchronize()


def test_temperature_error_paths():
    import torch
    n, k, g, seed = 3_000, 6.0, 3.0, 4
    p, a, R, r, t = _oracle_points(n, k, g, seed)
    rr = torch.from_numpy(r).cuda()
    tt = torch.from_numpy(t).cuda()
    idx = P.rhg_build_index(p, rr, tt)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    for bad in (0.0, -0.1, 1.0, float("nan")):
        with pytest.raises(P.RhgError) as e:
            P.rhg_temp_count_edges(idx, bad, row_ptr)
        assert e.value.status == 1
    # emit needs a temperature count at the same T
    P.rhg_count_edges(idx, row_ptr)
    col = torch.empty(int(row_ptr[-1].item()) + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(P.RhgError):
        P.rhg_temp_emit_edges(idx, 0.3, row_ptr, col)
    P.rhg_temp_count_edges(idx, 0.3, row_ptr)
    with pytest.raises(P.RhgError):
        P.rhg_temp_emit_edges(idx, 0.31, row_ptr, col)
    with pytest.raises(P.RhgError):  # and the threshold emit refuses it
        P.rhg_emit_edges(idx, row_ptr, col)
    nnz = int(row_ptr[-1].item())
    small = torch.empty(nnz - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(P.RhgError) as e:
        P.rhg_temp_emit_edges(idx, 0.3, row_ptr, small)
    assert e.value.status == 3
    full = torch.empty(nnz, dtype=torch.int32, device="cuda")
    P.rhg_temp_emit_edges(idx, 0.3, row_ptr, full, canonical_rows=True)
    orp, ocol, _, _ = O.temp_csr(r, t, R, 0.3, seed)
    assert np.array_equal(row_ptr.cpu().numpy(), orp)
    assert np.array_equal(full.cpu().numpy(), ocol)
    assert P.rhg_index_stats(idx)["ties"] == 0
    idx.free()
