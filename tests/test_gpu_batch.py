"""Batches: many uneven graphs captured into one HIP graph and launched as
one submission.  Every graph of a batch must equal, bit for bit (same
tuning, so the same row order), the same graph generated alone; the small
ones must match the oracle; overflowed graphs must be flagged and fixable;
and replays of the captured graph must give the same result each time."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from paper_1501_03545_amd import workloads as W
from gpu_util import oracle_check, pipeline_compare

pytestmark = pytest.mark.gpu

TUNINGS = [None, dict(band_width=1.0, cell_target=4, heavy_points=2048),
           dict(band_width=3.0, cell_target=1, heavy_points=16384),
           dict(band_width=1.5, cell_target=4, heavy_points=65536)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup_module(_):
    O.build(force=False)
    P.load()


def _alone(b):
    """The same graph through rhg_generate_async on the current stream."""
    import torch
    ref = P.GraphBuffers(b.params, b.tuning, col_capacity=b.col.numel())
    flag = torch.ones(1, dtype=torch.int32, device="cuda")
    P.rhg_generate_async(b.params, ref.r, ref.theta, ref.ws, ref.row_ptr, ref.col, flag, tuning=b.tuning)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    n, nnz = int(b.params.n), int(ref.row_ptr[-1].item())
    return (ref.r[:n].cpu().numpy(), ref.theta[:n].cpu().numpy(), ref.row_ptr.cpu().numpy(),
            ref.col[:nnz].cpu().numpy())


def _same(b, ref):
    n = int(b.params.n)
    nnz = int(b.row_ptr[-1].item())
    return (np.array_equal(b.r[:n].cpu().numpy(), ref[0]) and np.array_equal(b.theta[:n].cpu().numpy(), ref[1])
            and np.array_equal(b.row_ptr.cpu().numpy(), ref[2]) and np.array_equal(b.col[:nnz].cpu().numpy(), ref[3]))


def _bufs(draws, tunings, caps=None):
    out = []
    for g, d in enumerate(draws):
        p = P.rhg_plan(d["n"], d["avg_degree"], d["gamma"], d["seed"])
        cap = None if caps is None else caps.get(g)
        out.append(P.GraphBuffers(p, tunings[g % len(tunings)], col_capacity=cap))
    return out


def test_batch_equals_graphs_alone_and_oracle():
    import torch
    draws = W.batch_params(count=48, seed=4)
    bufs = _bufs(draws, TUNINGS)
    _say("batch of", len(bufs), "graphs, sum n", sum(d["n"] for d in draws))
    batch = P.Batch(bufs, n_streams=8)
    batch.launch()
    torch.cuda.synchronize()
    assert batch.fix_overflows() == []
    torch.cuda.synchronize()
    kinds = []
    for g, b in enumerate(bufs):
        assert _same(b, _alone(b)), "graph %d differs from the same graph generated alone" % g
        # every graph against the oracle: whole graphs up to n = 20000,
        # sampled rows against all points above
        _say("oracle", g, draws[g])
        kinds.append(oracle_check(O, b.graph(), draws[g]))
    _say("oracle checks", {k: kinds.count(k) for k in set(kinds)})
    assert kinds.count("full") >= 10


def test_batch_overflow_flags_and_replays():
    import torch
    draws = W.batch_params(count=12, seed=9)
    draws[3] = dict(n=0, avg_degree=5.0, gamma=2.5, seed=1)
    draws[7] = dict(n=2, avg_degree=0.5, gamma=2.5, seed=2)
    caps = {0: 8, 5: 8, 7: 0}
    bufs = _bufs(draws, TUNINGS, caps)
    refs = [None] * len(bufs)
    batch = P.Batch(bufs, n_streams=4)
    for rep in range(3):
        for b in bufs:  # eager work between replays
            b.row_ptr.fill_(-1)
            b.col.fill_(-7)
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        flags = batch.overflow[:len(bufs)].cpu().numpy()
        for g, b in enumerate(bufs):
            nnz = int(b.row_ptr[-1].item())
            assert flags[g] == (1 if nnz > batch.capacity[g] else 0), (rep, g, nnz)
        assert flags[0] == 1 and flags[5] == 1 and flags[3] == 0
        fixed = batch.fix_overflows()
        torch.cuda.synchronize()
        assert sorted(fixed) == sorted(np.nonzero(flags)[0].tolist())
        for g, b in enumerate(bufs):
            if refs[g] is None:
                refs[g] = _alone(b)
            assert _same(b, refs[g]), (rep, g)
        _say("replay", rep, "ok; overflowed", fixed)


def test_batch_rejects_empty_and_bad_graph():
    with pytest.raises(P.RhgError) as ei:
        P.Batch([])
    assert ei.value.status == P.RHG_EINVAL
    p = P.rhg_plan(1000, 6.0, 3.0, 1)
    b = P.GraphBuffers(p)
    b.ws = b.ws[:16]  # too small a workspace: rejected at capture, no batch
    with pytest.raises(P.RhgError):
        P.Batch([b])
