"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Edge sets are compared exactly (canonical rows), on the oracle's own points
for the search (index, count, scan, emit) and on each side's own points for
the whole pipeline (plan, sample and search)."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from gpu_util import canonical, check_simple_symmetric, pipeline_compare, run_search, ulp_diff

pytestmark = pytest.mark.gpu

C1 = (10_000, 6.0, 3.0)
C2 = (1_000_000, 10.0, 2.7)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _params_for(n, k, g, seed):
    if n >= 2:
        a, R = O.solve_R(n, k, g)
    else:
        a, R = (g - 1) / 2, 5.0
    return P.rhg_plan_radius(n, a, R, seed), a, R


@pytest.mark.parametrize("cfg", [C1, (100_000, 20.0, 2.2)])
def test_sampler_matches_oracle_bit_for_bit(cfg):
    import torch
    n, k, g = cfg
    _say("sampler", cfg)
    p = P.rhg_plan(n, k, g, 12345)
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    t = torch.empty(n, dtype=torch.float64, device="cuda")
    P.rhg_sample_points(p, r, t)
    ro, to, hard = O.sample(12345, p.alpha, p.R, n)
    assert hard == 0
    tg, rg = t.cpu().numpy(), r.cpu().numpy()
    assert np.array_equal(tg, to)  # Philox words and the angle product, bit for bit
    d = ulp_diff(rg, ro)
    _say("radius ulp differences: max", int(d.max()), "nonzero", int(np.count_nonzero(d)))
    assert np.array_equal(rg, ro)  # both sides round the radius correctly
    assert rg.min() >= 0 and rg.max() <= p.R


SMALL = [(2, 0.5, 2.5, 1), (3, 1.0, 2.5, 2), (17, 4.0, 2.5, 3), (1000, 64.0, 2.1, 4), (4097, 8.0, 3.5, 5),
         (2000, 30.0, 2.3, 6), C1 + (1,)]


@pytest.mark.parametrize("cfg", SMALL)
def test_search_parity_on_oracle_points(cfg):
    n, k, g, seed = cfg
    _say("search parity", cfg)
    params, a, R = _params_for(n, k, g, seed)
    r, t, _ = O.sample(seed, a, R, n)
    rp, col, stats = run_search(P, params, r, t)
    orp, ocol, nq, nt = O.csr(r, t, R)
    assert nt == 0 and stats["ties"] == 0
    assert np.array_equal(rp, orp)
    assert np.array_equal(canonical(rp, col), ocol)


def test_search_parity_independent_of_tuning():
    n, k, g = C1
    params, a, R = _params_for(n, k, g, 11)
    r, t, _ = O.sample(11, a, R, n)
    orp, ocol, _, _ = O.csr(r, t, R)
    for tun in [None, {"band_width": 0.25}, {"band_width": 3.0, "cell_target": 1},
                {"band_width": 0.5, "inner_radius": 12.0, "cell_target": 64}, {"cell_target": 2},
                {"band_width": 100.0}]:
        _say("tuning", tun)
        rp, col, stats = run_search(P, params, r, t, tuning=tun)
        assert np.array_equal(rp, orp)
        assert np.array_equal(canonical(rp, col), ocol)


def test_sweep_and_per_query_paths_give_the_same_rows():
    """A band of a wavefront is either swept (its union window staged in LDS,
    each lane binary-searching its own window) or searched per query (each
    lane's own window runs as one stream).  Forcing either path, and the
    sweep's linear filter instead of the binary search, gives the same rows
    entry for entry, across tunings, and the oracle's graph."""
    n, k, g = 20_000, 12.0, 2.3
    params, a, R = _params_for(n, k, g, 31)
    r, t, _ = O.sample(31, a, R, n)
    orp, ocol, _, _ = O.csr(r, t, R)
    for tun in [{}, {"band_width": 1.0, "heavy_points": 2048}, {"band_width": 3.0, "cell_target": 4}]:
        rp_s, col_s, st_s = run_search(P, params, r, t, tuning=dict(tun) or None)
        # every union swept (huge sweep_max), none swept unless windows overlap
        rp_w, col_w, st_w = run_search(P, params, r, t, tuning=dict(tun, sweep_max=1 << 30))
        rp_q, col_q, st_q = run_search(P, params, r, t, tuning=dict(tun, sweep_max=-1))
        # a mix: short unions swept, long ones per query
        rp_m, col_m, st_m = run_search(P, params, r, t, tuning=dict(tun, sweep_max=24))
        # swept chunks filtered candidate by candidate
        rp_l, col_l, st_l = run_search(P, params, r, t, tuning=dict(tun, sweep_linear=1))
        # per-query candidate streams read through registers, never staged in LDS
        rp_r, col_r, _ = run_search(P, params, r, t, tuning=dict(tun, sweep_max=-1, no_stream_stage=1))
        _say("paths", tun, st_s, st_w, st_q, st_m)
        assert st_w["swept"] >= st_s["swept"] > st_m["swept"] > st_q["swept"]
        # the linear filter and the binary search test the same candidates
        assert st_l["tests"] == st_s["tests"]
        for rp_x in (rp_s, rp_w, rp_q, rp_l, rp_r, rp_m):
            assert np.array_equal(rp_x, orp)
        # the same tested pairs in the same order: the same bytes
        assert np.array_equal(col_s, col_l)
        assert np.array_equal(col_q, col_r)
        # rows staged by the count pass and copied by the emit pass, with
        # slots large enough and with slots too small for most rows (those
        # wavefronts searched again): the same bytes
        for st in ({"stage": 1}, {"stage": 1, "stage_pct": 1}):
            rp_x, col_x, _ = run_search(P, params, r, t, tuning=dict(tun, **st))
            assert np.array_equal(rp_x, rp_s) and np.array_equal(col_x, col_s), st
        for rp_x, col_x in ((rp_s, col_s), (rp_w, col_w), (rp_q, col_q), (rp_m, col_m)):
            assert np.array_equal(canonical(rp_x, col_x), ocol)


def test_crowded_sector_long_streams():
    """Points crowded into a narrow sector give long per-query streams: the
    longest (over 4096 entries) take the register path even by default; with
    no_stream_stage every stream does.  Both match the oracle."""
    n, k, g = 8_000, 8.0, 2.6
    params, a, R = _params_for(n, k, g, 41)
    r, t, _ = O.sample(41, a, R, n)
    t = t.copy()
    t[: n // 2] = t[: n // 2] * 1e-3  # half the points within 0.0063 rad
    orp, ocol, _, nt = O.csr(r, t, R)
    rp_s, col_s, st_s = run_search(P, params, r, t, tuning={"sweep_max": -1})
    rp_r, col_r, st_r = run_search(P, params, r, t, tuning={"sweep_max": -1, "no_stream_stage": 1})
    rp_d, col_d, st_d = run_search(P, params, r, t)
    _say("crowded", st_s, "register path only:", st_r, "default:", st_d)
    assert st_s["register_streams"] > 0
    assert st_r["register_streams"] > st_s["register_streams"]
    for rp_x, col_x in ((rp_s, col_s), (rp_r, col_r), (rp_d, col_d)):
        assert np.array_equal(rp_x, orp)
        assert np.array_equal(canonical(rp_x, col_x), ocol)
    assert np.array_equal(col_r, col_s)


def test_search_degenerate_inputs():
    """Points at the origin, on the rim, sharing an angle, duplicated, and
    straddling the 0 / 2 pi seam."""
    n, k, g = 3000, 10.0, 2.5
    params, a, R = _params_for(n, k, g, 21)
    r, t, _ = O.sample(21, a, R, n)
    r = r.copy(); t = t.copy()
    r[0] = 0.0
    r[1] = R
    r[2], t[2] = r[3], t[3]                      # duplicate point
    t[4:40] = t[40]                              # many equal angles
    t[41] = 0.0
    t[42] = np.nextafter(2 * np.pi, 0)           # largest double below 2 pi
    t[43] = 1e-12
    r[41:44] = R - 0.1
    rp, col, stats = run_search(P, params, r, t)
    orp, ocol, _, nt = O.csr(r, t, R)
    # the origin and the rim point are exactly R apart: a true tie, which
    # both sides must resolve as an edge (distance <= R)
    assert nt > 0 and stats["ties"] > 0
    assert np.array_equal(rp, orp)
    assert np.array_equal(canonical(rp, col), ocol)
    # staged: the same bytes
    rp1, col1, _ = run_search(P, params, r, t, tuning={"stage": 1})
    assert np.array_equal(rp1, rp) and np.array_equal(col1, col)
    assert rp[1] - rp[0] == n - 1  # the origin sees every vertex
    assert 0 in col[rp[1]:rp[2]]


def test_empty_and_tiny_graphs():
    import torch
    for n in [0, 1]:
        p = P.rhg_plan(n, 5.0, 2.5, 1)
        g = P.rhg_generate(n, 5.0, 2.5, 1)
        assert g.nnz == 0
        assert g.row_ptr.cpu().tolist() == [0] * (n + 1)


def test_staged_tiny_and_ragged_graphs():
    """Staged counts on graphs of one to a few wavefronts, ragged tails
    included, with slots that fit, slots too small (every such wavefront
    searched again) and no heavy set: the oracle's edge set, and the same
    bytes as the unstaged passes of the same tuning."""
    a = 0.75
    for n in (1, 2, 63, 64, 65, 129, 700):
        R = 2.0 * math.log(max(n, 2)) + 3.0
        params = P.rhg_plan_radius(n, a, R, 5)
        r, t, _ = O.sample(5, a, R, n)
        orp, ocol, _, nt = O.csr(r, t, R)
        assert nt == 0
        for tu in ({}, {"heavy_points": 1}, {"stage_pct": 1}):
            rp, col, st = run_search(P, params, r, t, tuning=dict(tu, stage=1))
            rp0, col0, _ = run_search(P, params, r, t, tuning=dict(tu, stage=-1))
            assert st["staged_waves"] > 0, (n, tu)
            assert np.array_equal(rp, orp), (n, tu)
            assert np.array_equal(rp, rp0) and np.array_equal(col, col0), (n, tu)
            assert np.array_equal(canonical(rp, col), ocol), (n, tu)


def test_invalid_points_and_capacity_are_reported():
    import torch
    n = 100
    params, a, R = _params_for(n, 5.0, 2.5, 1)
    r, t, _ = O.sample(1, a, R, n)
    bad = r.copy()
    bad[7] = R * 1.5
    with pytest.raises(P.RhgError) as ei:
        run_search(P, params, bad, t)
    assert ei.value.status == P.RHG_EINVAL
    rt = torch.from_numpy(r).cuda()
    tt = torch.from_numpy(t).cuda()
    idx = P.rhg_build_index(params, rt, tt)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    P.rhg_count_edges(idx, row_ptr)
    nnz = int(row_ptr[-1])
    assert nnz > 0
    small = torch.empty(nnz - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(P.RhgError) as ei:
        P.rhg_emit_edges(idx, row_ptr, small)
    assert ei.value.status == P.RHG_ECAPACITY


def test_generate_pipeline_matches_oracle_c1():
    n, k, g_ = C1
    _say("generate C1")
    g = P.rhg_generate(n, k, g_, 1)
    a, R, r_o, t_o, orp, ocol, st = O.generate(n, k, g_, 1)
    assert g.params.R == R and g.params.alpha == a
    assert st["ties"] == 0
    mism = pipeline_compare(g, r_o, t_o, R, orp, ocol)
    _say("pipeline mismatched pairs", mism)
    assert mism == 0


def test_c2_full_graph_invariants_and_sampled_rows():
    n, k, g_ = C2
    _say("generate C2")
    g = P.rhg_generate(n, k, g_, 2)
    rp = g.row_ptr.cpu().numpy()
    col = g.col_idx.cpu().numpy()
    check_simple_symmetric(rp, col)
    deg = np.diff(rp)
    _say("C2 edges", col.size // 2, "mean degree", deg.mean())
    a, R = O.solve_R(n, k, g_)
    r_o, t_o, hard = O.sample(2, a, R, n)
    assert hard == 0
    assert np.array_equal(g.theta.cpu().numpy(), t_o)
    assert np.array_equal(g.r.cpu().numpy(), r_o)
    # rows stratified by radius quantile, plus the 32 largest degrees
    order = np.argsort(r_o)
    strat = order[np.linspace(0, n - 1, 160).astype(np.int64)]
    top = np.argsort(deg)[-32:]
    which = np.unique(np.concatenate([strat, top]))
    ptr, ocol, _, nt = O.rows(r_o, t_o, R, which)
    assert nt == 0
    for a_, i in enumerate(which):
        assert np.array_equal(np.sort(col[rp[i]:rp[i + 1]]), ocol[ptr[a_]:ptr[a_ + 1]]), i
    # the GPU search on the oracle's own points is bit-exact on the same rows
    rp2, col2, stats = run_search(P, P.rhg_plan_radius(n, a, R, 2), r_o, t_o)
    assert stats["ties"] == 0
    for a_, i in enumerate(which):
        assert np.array_equal(np.sort(col2[rp2[i]:rp2[i + 1]]), ocol[ptr[a_]:ptr[a_ + 1]])
    # the plain binary64 path (no FP32 screen), as this configuration names
    # it, gives the same graph entry for entry
    rp3, col3, st3 = run_search(P, P.rhg_plan_radius(n, a, R, 2), r_o, t_o, tuning={"fp64_only": 1})
    assert st3["fp32_undecided"] == 0 and stats["fp32_undecided"] > 0
    assert np.array_equal(rp3, rp2) and np.array_equal(col3, col2)
    # per-query candidate streams through registers only (the path of the
    # longest streams) instead of the LDS stage: the same bytes
    rp4, col4, _ = run_search(P, P.rhg_plan_radius(n, a, R, 2), r_o, t_o, tuning={"no_stream_stage": 1})
    assert np.array_equal(rp4, rp2) and np.array_equal(col4, col2)
    # rows counted and searched again instead of staged (staging is the
    # default from n = 2^19): the same bytes
    rp5, col5, _ = run_search(P, P.rhg_plan_radius(n, a, R, 2), r_o, t_o, tuning={"stage": -1})
    assert np.array_equal(rp5, rp2) and np.array_equal(col5, col2)


def test_c3_full_size_points_and_sampled_rows():
    """n = 1e8, average degree 20, gamma 2.2, through the calls and launch
    configuration the benchmark times: every angle and radius against the
    oracle's, bit for bit, and sampled rows (innermost and outermost points,
    radius quantiles, the largest degrees, random) against brute force over
    all 1e8 points."""
    import torch
    from paper_1501_03545_amd import workloads as W
    cfg = W.LARGE
    n, k, g_, seed = cfg["n"], cfg["avg_degree"], cfg["gamma"], cfg["seed"]
    p = P.rhg_plan(n, k, g_, seed)
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    t = torch.empty(n, dtype=torch.float64, device="cuda")
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ws = torch.empty(P.rhg_index_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    P.rhg_sample_points(p, r, t)
    idx = P.rhg_build_index(p, r, t, workspace=ws, validate=False)
    P.rhg_count_edges(idx, row_ptr)
    nnz = int(row_ptr[-1].item())
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    P.rhg_emit_edges(idx, row_ptr, col)
    stats = P.rhg_index_stats(idx)
    idx.free()
    del ws
    _say("C3 edges", nnz // 2, stats)
    assert stats["ties"] == 0
    rg, tg = r.cpu().numpy(), t.cpu().numpy()
    deg = torch.diff(row_ptr).cpu().numpy()
    a, R = O.solve_R(n, k, g_)
    assert (a, R) == (p.alpha, p.R)
    r_o, t_o, hard = O.sample(seed, a, R, n)
    _say("oracle sampled", hard)
    assert hard == 0
    assert np.array_equal(tg, t_o)
    assert np.array_equal(rg, r_o)
    # 512 rows stratified by radius quantile, the 32 innermost points (the
    # hubs), the 32 largest degrees and 32 random rows, each against all 1e8
    # points by brute force
    rng = np.random.default_rng(33)
    order = np.argsort(r_o, kind="stable")
    strat = order[np.linspace(0, n - 1, 512).astype(np.int64)]
    inner = order[:32]
    top = np.argpartition(deg, -32)[-32:]
    which = np.unique(np.concatenate([strat, inner, top, rng.integers(0, n, 32)]).astype(np.int64))
    del order
    _say("C3 brute-force rows", len(which))
    ptr, ocol, _, nt = O.rows(r_o, t_o, R, which)
    assert nt == 0
    rp = row_ptr.cpu().numpy()
    for a_, i in enumerate(which):
        mine = np.sort(col[rp[i]:rp[i + 1]].cpu().numpy())
        assert np.array_equal(mine, ocol[ptr[a_]:ptr[a_ + 1]]), (i, deg[i])
    _say("C3 rows checked", len(which), "entries", int(ptr[-1]), "max degree", int(deg[which].max()))


def test_count_and_emit_twice_on_one_index():
    """Counting and emitting a second time on the same index gives the same
    bytes and the same per-pass test count."""
    import torch
    n, k, g = 30_000, 16.0, 2.4
    params, a, R = _params_for(n, k, g, 77)
    r, t, _ = O.sample(77, a, R, n)
    idx = P.rhg_build_index(params, torch.from_numpy(r).cuda(), torch.from_numpy(t).cuda())
    out = []
    for _ in range(2):
        rp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        P.rhg_count_edges(idx, rp)
        nnz = int(rp[-1].item())
        col = torch.empty(nnz, dtype=torch.int32, device="cuda")
        P.rhg_emit_edges(idx, rp, col)
        torch.cuda.synchronize()
        out.append((rp.cpu().numpy(), col.cpu().numpy(), P.rhg_index_stats(idx)))
    idx.free()
    _say("twice:", out[0][2], out[1][2])
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2]["tests"] > 0 and out[1][2]["tests"] == out[0][2]["tests"]
    orp, ocol, _, _ = O.csr(r, t, R)
    assert np.array_equal(out[1][0], orp) and np.array_equal(canonical(out[1][0], out[1][1]), ocol)
