"""A seeded sweep of random graphs and tunings: the HIP search through the C
ABI, on the oracle's own points, against the oracle's CSR entry for entry
(rows canonicalised), at sizes the oracle's all-pairs definition finishes in
about a second.  Parameters span the batch mix (gamma 2.1 .. 3.5, average
degree 4 .. 64) at n = 500 .. 20000, and every tuning switch the library
has; each case prints its parameters before it runs."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P
from gpu_util import canonical, check_simple_symmetric, run_search

pytestmark = pytest.mark.gpu

TUNINGS = [None, {"band_width": 0.5}, {"band_width": 3.0}, {"cell_target": 8}, {"heavy_points": 256},
           {"no_stream_stage": 1, "sweep_max": -1}, {"fp64_only": 1}, {"sweep_max": 1 << 30}, {"sweep_linear": 1},
           {"exact_inline": 1}, {"defer_cap": 1},
           {"band_width": 1.0, "cell_target": 2, "heavy_points": 1024},
           {"stage": 1}, {"stage": 1, "stage_pct": 1}, {"stage": 1, "defer_cap": 1}, {"stage": 1, "exact_inline": 1},
           {"stage": 1, "fp64_only": 1}, {"stage": 1, "band_width": 0.5, "stage_pct": 20, "heavy_points": 64}]


def _cases(count=20, seed=20261202):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(10 ** rng.uniform(2.7, 4.3)))
        g = float(2.1 + 1.4 * rng.random())
        k = float(4.0 + (min(64.0, n / 20.0) - 4.0) * rng.random())
        out.append((n, k, g, int(rng.integers(0, 2**62)), TUNINGS[i % len(TUNINGS)]))
    return out


CASES = _cases()


def setup_module(_):
    O.build(force=False)
    P.load()


@pytest.mark.parametrize("case", CASES, ids=["n%d_k%.1f_g%.2f_%d" % (c[0], c[1], c[2], i) for i, c in enumerate(CASES)])
def test_random_graph_matches_oracle(case):
    n, k, g, seed, tun = case
    print("case", case, flush=True)
    sys.stdout.flush()
    a, R = O.solve_R(n, k, g)
    r, t, hard = O.sample(seed, a, R, n)
    assert hard == 0
    orp, ocol, _, _ = O.csr(r, t, R)
    rp, col, st = run_search(P, P.rhg_plan_radius(n, a, R, seed), r, t, tuning=tun)
    assert st["ties"] == 0
    check_simple_symmetric(rp, col)
    assert np.array_equal(rp, orp)
    assert np.array_equal(canonical(rp, col), ocol)
