"""The near-threshold pair constructor used by the GPU exactness tests lands
each pair on the intended side of the threshold, within 2^-k of it, as the
oracle's binary128 decision and a 60-digit evaluation agree (CPU)."""
import numpy as np
import pytest

import adversarial as ADV


@pytest.mark.parametrize("cfg", [(10_000, 6.0, 3.0, 1), (100_000_000, 20.0, 2.2, 3)])
def test_constructed_pairs_sides(cfg):
    import oracle
    import paper_1501_03545_amd as P

    p0 = P.rhg_plan(*cfg)
    tuning = {"inner_radius": max(0.0, p0.R - np.log(cfg[0]) / p0.alpha)}
    E = P.rhg_layout_bands(P.rhg_plan_radius(1000, p0.alpha, p0.R, 0), tuning)
    assert E[0] == 0.0 and E[-1] == p0.R and all(a < b for a, b in zip(E, E[1:]))
    pairs = ADV.constructed_pairs(p0.R, tuple(E), 0)
    kinds = {p[0] for p in pairs}
    assert kinds == {"pi", "mid", "rim", "edge", "cell", "seam", "tie"}
    for kind, k, side, r1, t1, r2, t2 in pairs:
        assert 0.0 <= r1 <= p0.R and 0.0 <= r2 <= p0.R
        assert 0.0 <= t1 < ADV.TWO_PI_D and 0.0 <= t2 < ADV.TWO_PI_D
        e = oracle.is_edge_quad(r1, t1, r2, t2, p0.R)
        if side == 0:
            assert e, (kind, r1, t1, r2, t2)
            continue
        off = ADV.rel_offset(p0.R, r1, t1, r2, t2)
        if k <= 36:
            assert e == (side < 0), (kind, k, side, off)
            assert (off < 0) == (side < 0)
        if kind in ("pi", "rim", "mid"):
            assert abs(off) < 2.0 ** -(k - 2), (kind, k, off)
