"""GPU parity of the dynamic model: after every batch of moves the state's
graph must equal the oracle's brute force on the moved points, entry for
entry (ascending rows).  Covers single moves, small and large batches, all
vertices at once, moves across bands, the seam and the centre, a larger
graph checked on the rows a step rewrites, and refused batches."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from paper_1501_03545_amd import workloads as W
from gpu_util import check_simple_symmetric

pytestmark = pytest.mark.gpu

TWO_PI_D = 6.283185307179586


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _start(n, k, g, seed, tuning=None, share=1e30):
    """A state on the oracle's points; by default every batch is applied
    incrementally (share 1e30), the path under test."""
    import torch
    a, R = O.solve_R(n, k, g)
    r, t, hard = O.sample(seed, a, R, n)
    assert hard == 0
    p = P.rhg_plan_radius(n, a, R, seed)
    d = P.DynGraph(p, torch.from_numpy(r).cuda(), torch.from_numpy(t).cuda(), tuning=tuning)
    d.set_regenerate_share(share)
    return d, R, r, t


def _move(d, ids, rn, tn):
    import torch
    d.move(torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int32)).cuda(),
           torch.from_numpy(np.ascontiguousarray(rn, dtype=np.float64)).cuda(),
           torch.from_numpy(np.ascontiguousarray(tn, dtype=np.float64)).cuda())


def _check_full(d, R, r, t, allow_ties=False):
    """The state's graph against the oracle's; constructed points may sit
    exactly at distance R (a point at the centre and one on the rim): the
    oracle counts such pairs as ties and joins them, as the library does."""
    G = d.graph()
    assert np.array_equal(G.r.cpu().numpy(), r) and np.array_equal(G.theta.cpu().numpy(), t)
    orp, ocol, _, ties = O.csr(r, t, R)
    assert allow_ties or ties == 0
    rp = G.row_ptr.cpu().numpy()
    assert np.array_equal(rp, orp)
    assert np.array_equal(G.col_idx.cpu().numpy(), ocol)


@pytest.mark.parametrize("cfg", [(20_000, 10.0, 2.5, 1, 1e30), (8_000, 30.0, 2.1, 2, 1e30), (12_000, 6.0, 3.0, 3, 1e30),
                                 (20_000, 10.0, 2.5, 1, 0.125), (9_000, 8.0, 2.6, 4, 0.0)])
def test_moves_keep_the_graph_equal_to_regeneration(cfg):
    """Incremental steps (share 1e30), the default policy (some steps
    regenerate) and regeneration only (share 0)."""
    n, k, g, seed, share = cfg
    d, R, r, t = _start(n, k, g, seed, share=share)
    _check_full(d, R, r, t)
    rng = np.random.default_rng(seed)
    for step, kk in enumerate([1, 7, 100, 1000, n // 4, n]):
        ids, rn, tn = W.move_batch(rng, r, t, kk, R, angle_step=0.02 * (step + 1), radius_step=0.3)
        _say("step", step, "moves", kk)
        _move(d, ids, rn, tn)
        r, t = O.apply_moves(r, t, ids, rn, tn)
        _check_full(d, R, r, t)
        st = d.last_step()
        assert st["changed_rows"] >= kk
        if share == 0.0:
            assert st["changed_rows"] == n
    d.close()


def test_moves_to_the_centre_the_rim_and_across_the_seam():
    n, k, g, seed = 10_000, 8.0, 2.4, 5
    d, R, r, t = _start(n, k, g, seed)
    rng = np.random.default_rng(9)
    ids = rng.choice(n, size=12, replace=False).astype(np.int32)
    rn = np.array([0.0, 1e-3, R, R, R * 0.5, R - 1e-12, 0.0, R * 0.9, R * 0.9, 2.0, R, 0.5])
    tn = np.array([0.0, 3.0, 0.0, TWO_PI_D - 1e-15, 1e-15, np.pi, 6.0, 0.0, 6.28318530717958, 1.0, 3.0, 5.0])
    _move(d, ids, rn, tn)
    r, t = O.apply_moves(r, t, ids, rn, tn)
    _check_full(d, R, r, t, allow_ties=True)
    # and back, plus a vertex that does not move at all (same coordinates)
    ids2 = np.concatenate([ids, [int(np.setdiff1d(np.arange(n), ids)[0])]]).astype(np.int32)
    rn2 = np.concatenate([R * rng.random(12), [r[ids2[-1]]]])
    tn2 = np.concatenate([TWO_PI_D * rng.random(12), [t[ids2[-1]]]])
    _move(d, ids2, rn2, tn2)
    r, t = O.apply_moves(r, t, ids2, rn2, tn2)
    _check_full(d, R, r, t)
    d.close()


def test_tunings_and_repeated_steps():
    n, k, g, seed = 15_000, 12.0, 2.3, 7
    for tu in (None, {"band_width": 0.7}, {"fp64_only": 1}, {"cell_target": 4, "heavy_points": 64}):
        d, R, r, t = _start(n, k, g, seed, tuning=tu)
        rng = np.random.default_rng(11)
        for _ in range(5):
            ids, rn, tn = W.move_batch(rng, r, t, 300, R, angle_step=0.05, radius_step=0.5)
            _move(d, ids, rn, tn)
            r, t = O.apply_moves(r, t, ids, rn, tn)
        _check_full(d, R, r, t)
        d.close()


def test_n1e6_steps_against_the_oracle_rows():
    """The n = 1e6, average degree 10, gamma = 2.7 graph: three steps of 2000
    moves; after each, the rows the step rewrote (sampled) and random rows
    against all n points, plus the whole CSR's symmetry."""
    n, k, g, seed = 1_000_000, 10.0, 2.7, 2
    d, R, r, t = _start(n, k, g, seed)
    rng = np.random.default_rng(13)
    for step in range(3):
        ids, rn, tn = W.move_batch(rng, r, t, 2000, R, angle_step=0.01, radius_step=0.2)
        _move(d, ids, rn, tn)
        r, t = O.apply_moves(r, t, ids, rn, tn)
        G = d.graph()
        rp = G.row_ptr.cpu().numpy()
        col = G.col_idx.cpu().numpy()
        check_simple_symmetric(rp, col)
        # moved rows, rows that held a moved vertex, random rows
        nbr = np.unique(np.concatenate([col[rp[i]:rp[i + 1]] for i in ids[:40]]))
        which = np.unique(np.concatenate([ids[:60], nbr[:60], rng.choice(n, 60, replace=False)])).astype(np.int64)
        ptr, ocol, _, nt = O.rows(r, t, R, which)
        assert nt == 0
        for j, i in enumerate(which):
            assert np.array_equal(col[rp[i]:rp[i + 1]], ocol[ptr[j]:ptr[j + 1]]), (step, i)
        _say("step", step, d.last_step(), "edges", int(rp[-1]) // 2)
    d.close()


def test_refused_batches_leave_the_state_unchanged():
    n, k, g, seed = 5_000, 8.0, 2.5, 4
    d, R, r, t = _start(n, k, g, seed)
    bad = [
        (np.array([1, 2, 1]), np.array([1.0, 2.0, 3.0]), np.array([0.1, 0.2, 0.3])),   # duplicate
        (np.array([1, n]), np.array([1.0, 2.0]), np.array([0.1, 0.2])),                # id out of range
        (np.array([1, -1]), np.array([1.0, 2.0]), np.array([0.1, 0.2])),
        (np.array([3]), np.array([R * 1.0001]), np.array([0.5])),                      # outside the disk
        (np.array([3]), np.array([1.0]), np.array([TWO_PI_D])),                        # angle 2 pi
        (np.array([3]), np.array([float("nan")]), np.array([0.5])),
    ]
    for ids, rn, tn in bad:
        with pytest.raises(P.RhgError) as e:
            _move(d, ids, rn, tn)
        assert e.value.status == P.RHG_EINVAL
    _check_full(d, R, r, t)
    # a valid batch after the refusals
    ids, rn, tn = W.move_batch(np.random.default_rng(3), r, t, 50, R)
    _move(d, ids, rn, tn)
    r, t = O.apply_moves(r, t, ids, rn, tn)
    _check_full(d, R, r, t)
    d.close()
