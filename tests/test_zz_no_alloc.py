"""rhg_generate_async_noalloc (the library's own per-GPU workspace, no device
allocation) against rhg_generate_async on caller workspace: the same points
and the same CSR, bit for bit, on two calls in a row (the second graph
smaller than the first, so stale contents of the shared array would show),
the smaller one also against the oracle; a graph too large for the array is
refused."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from gpu_util import pipeline_compare

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _buffers(p):
    import torch
    n = max(int(p.n), 1)
    cap = P.expected_col_capacity(p)
    return dict(r=torch.empty(n, dtype=torch.float64, device="cuda"),
                theta=torch.empty(n, dtype=torch.float64, device="cuda"),
                row_ptr=torch.empty(int(p.n) + 1, dtype=torch.int64, device="cuda"),
                col=torch.empty(cap, dtype=torch.int32, device="cuda"),
                flag=torch.zeros(1, dtype=torch.int32, device="cuda"))


def test_noalloc_equals_workspace_path_on_two_calls():
    import torch
    P.load()
    for (n, k, g, seed) in ((200_000, 12.0, 2.4, 5), (30_000, 8.0, 2.8, 6)):
        p = P.rhg_plan(n, k, g, seed)
        _say("[noalloc] n=%d k=%g gamma=%g seed=%d workspace=%d bytes" % (n, k, g, seed,
                                                                       P.rhg_index_workspace_bytes(p)))
        a = _buffers(p)
        ws = torch.empty(P.rhg_index_workspace_bytes(p), dtype=torch.uint8, device="cuda")
        P.rhg_generate_async(p, a["r"], a["theta"], ws, a["row_ptr"], a["col"], a["flag"])
        b = _buffers(p)
        P.rhg_generate_async_noalloc(p, b["r"], b["theta"], b["row_ptr"], b["col"], b["flag"])
        torch.cuda.synchronize()
        assert int(a["flag"].item()) == 0 and int(b["flag"].item()) == 0
        nnz = int(a["row_ptr"][-1].item())
        assert torch.equal(a["row_ptr"], b["row_ptr"])
        assert torch.equal(a["col"][:nnz], b["col"][:nnz])
        assert torch.equal(a["r"], b["r"]) and torch.equal(a["theta"], b["theta"])
        _say("[noalloc] same bytes: m=%d" % (nnz // 2))
        if n <= 30_000:
            _, R, r_o, t_o, orp, ocol, st = O.generate(n, k, g, seed)
            assert st["ties"] == 0
            gr = P.Graph(params=p, row_ptr=b["row_ptr"], col_idx=b["col"][:nnz], r=b["r"], theta=b["theta"])
            assert pipeline_compare(gr, r_o, t_o, R, orp, ocol) == 0
        del ws


def test_noalloc_refuses_a_graph_larger_than_its_array():
    p = P.rhg_plan(2_000_000, 10.0, 2.5, 1)
    assert P.rhg_index_workspace_bytes(p) > P.NOALLOC_SCRATCH_BYTES
    b = _buffers(P.rhg_plan(1000, 10.0, 2.5, 1))
    with pytest.raises(P.RhgError) as ei:
        P.rhg_generate_async_noalloc(p, b["r"], b["theta"], b["row_ptr"], b["col"], b["flag"])
    assert ei.value.status == P.RHG_ECAPACITY
