"""Pins for the oracle's temperature model (the distance-dependent connection
probability that Sec. 2.1 sets aside), against what the definition and the
mathematics fix rather than against the oracle itself:

* the decision u < p(d) on constructed pairs near the boundary, against the
  definition evaluated in 60-digit arithmetic on the hyperbolic distance of
  Eq. (2) (the Poincare metric, an independent form of the distance);
* the limit T -> 0, where the model is the threshold rule d <= R: every pair
  on which the two oracles disagree lies in the narrow shell that the
  coin's resolution allows;
* edge frequencies against p(d) over all pairs of a graph (binomial test per
  probability bin);
* the mean degree over seeds against an independent numerical integration
  of the model's expected degree;
* the coins: symmetric in the pair, uniform on (0, 1].
CPU only.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

import oracle as O
from quadrature import expected_degree_temperature

TWO_PI_D = 6.283185307179586
C1 = (10_000, 6.0, 3.0)
C3 = (100_000_000, 20.0, 2.2)
TWO53 = 1 << 53


def setup_module(_):
    O.build(force=False)


def _mp_dist_poincare(r1, t1, r2, t2):
    """Eq. (2) on the points mapped by mapToPoincare (Appendix B.2)."""
    def to_disk(r, t):
        rr = mp.sqrt((mp.cosh(r) - 1) / (mp.cosh(r) + 1))
        return rr * mp.cos(t), rr * mp.sin(t), rr
    x1, y1, n1 = to_disk(mp.mpf(r1), mp.mpf(t1))
    x2, y2, n2 = to_disk(mp.mpf(r2), mp.mpf(t2))
    d2 = (x1 - x2) ** 2 + (y1 - y2) ** 2
    return mp.acosh(1 + 2 * d2 / ((1 - n1**2) * (1 - n2**2)))


def _mp_edge(r1, t1, r2, t2, R, T, a):
    """The definition, literally: u = a 2^-53 < 1 / (1 + e^{(d - R)/(2T)})."""
    d = _mp_dist_poincare(r1, t1, r2, t2)
    p = 1 / (1 + mp.exp((d - mp.mpf(R)) / (2 * mp.mpf(T))))
    return mp.mpf(a) / mp.mpf(TWO53) < p


def _pairs_near_boundary(R, T, rng, count):
    """Pairs whose distance is within a relative 2^-k (k = 8 .. 44) of the
    coin's boundary D(u) = R + 2T ln((1 - u)/u), with coins drawn at random
    and at the extremes (u near 2^-53, 1/2 and 1)."""
    out = []
    specials = [1, 2, TWO53 // 2 - 1, TWO53 // 2, TWO53 // 2 + 1, TWO53 - 2, TWO53 - 1]
    draws = 0
    while len(out) < count:
        a = specials[draws] if draws < len(specials) else int(rng.integers(1, TWO53))
        draws += 1
        u = mp.mpf(a) / TWO53
        D = mp.mpf(R) + 2 * mp.mpf(T) * mp.log((1 - u) / u)
        for _ in range(64):   # radius pairs whose distances can reach D (none may exist)
            r1 = float(R * rng.random() ** 0.3)
            r2 = float(R * rng.random() ** 0.3)
            lo, hi = abs(r1 - r2), r1 + r2
            k = int(rng.integers(8, 45))
            target = D * (1 + (1 if rng.random() < 0.5 else -1) * mp.mpf(2) ** (-k))
            if not (lo < target < hi):
                continue
            c = (mp.cosh(target) - mp.cosh(mp.mpf(r1) - mp.mpf(r2))) / (2 * mp.sinh(r1) * mp.sinh(r2))
            dth = float(2 * mp.asin(mp.sqrt(c)))
            t1 = TWO_PI_D * rng.random()
            t2 = t1 + dth
            if t2 >= TWO_PI_D:
                t2 -= TWO_PI_D
            if 0.0 <= t2 < TWO_PI_D:
                out.append((r1, t1, r2, t2, a))
                break
    return out


@pytest.mark.parametrize("cfg", [C1, C3])
@pytest.mark.parametrize("T", [0.05, 0.4, 0.9])
def test_decision_equals_the_definition_in_60_digits(cfg, T):
    mp.mp.dps = 60
    _, R = O.solve_R(*cfg)
    rng = np.random.default_rng(int(T * 1000) + cfg[0] % 97)
    quad = 0
    for (r1, t1, r2, t2, a) in _pairs_near_boundary(R, T, rng, 80):
        ref = _mp_edge(r1, t1, r2, t2, R, T, a)
        e, q, ties = O.temp_is_edge(r1, t1, r2, t2, R, T, a)
        assert ties == 0
        assert e == ref, (r1, t1, r2, t2, a)
        assert O.temp_is_edge(r2, t2, r1, t1, R, T, a)[0] == e
        assert O.temp_is_edge_quad(r1, t1, r2, t2, R, T, a) == ref
        quad += q
    assert quad > 0  # the binary128 stage was reached


def test_decision_special_coins_and_points():
    _, R = O.solve_R(*C1)
    T = 0.3
    # u = 1 (a = 2^53) is never below p(d) < 1, even for a point and itself
    assert not O.temp_is_edge(1.0, 0.5, 1.0, 0.5, R, T, TWO53)[0]
    # identical points: d = 0 and p(0) = 1 / (1 + e^{-R/(2T)}), just below 1
    p0 = 1.0 / (1.0 + math.exp(-R / (2 * T)))
    a_below = int(p0 * TWO53) - 4
    assert O.temp_is_edge(2.0, 1.0, 2.0, 1.0, R, T, a_below)[0]
    # the smallest coin, u = 2^-53: an edge iff d < R + 2T ln(2^53 - 1)
    rho = R + 2 * T * math.log(TWO53 - 1)
    r = rho / 2
    assert O.temp_is_edge(r * (1 - 1e-6), 0.0, r * (1 - 1e-6), math.pi, R, T, 1)[0]
    assert not O.temp_is_edge(r * (1 + 1e-6), 0.0, r * (1 + 1e-6), math.pi, R, T, 1)[0]
    # u = 1/2: p(d) > 1/2 iff d < R
    assert O.temp_is_edge(R / 2 * (1 - 1e-9), 0.0, R / 2 * (1 - 1e-9), math.pi, R, T, TWO53 // 2)[0]
    assert not O.temp_is_edge(R / 2 * (1 + 1e-9), 0.0, R / 2 * (1 + 1e-9), math.pi, R, T, TWO53 // 2)[0]


def _distances(r, t):
    """Pairwise hyperbolic distances (i < j) in binary64 from the
    non-negative form, for the statistics below."""
    n = r.shape[0]
    i, j = np.triu_indices(n, 1)
    dth = np.abs(t[i] - t[j])
    dth = np.minimum(dth, 2 * np.pi - dth)
    ch = np.cosh(r[i] - r[j]) + 2 * np.sinh(r[i]) * np.sinh(r[j]) * np.sin(dth / 2) ** 2
    return i, j, np.arccosh(ch)


def test_vanishing_temperature_gives_the_threshold_graph():
    n, k, g = 2500, 6.0, 2.6
    a, R = O.solve_R(n, k, g)
    r, t, _ = O.sample(7, a, R, n)
    T = 1e-4
    rp0, c0, _, _ = O.csr(r, t, R)
    rp1, c1, _, ties = O.temp_csr(r, t, R, T, 7)
    assert ties == 0
    e0 = set(zip(np.repeat(np.arange(n), np.diff(rp0)).tolist(), c0.tolist()))
    e1 = set(zip(np.repeat(np.arange(n), np.diff(rp1)).tolist(), c1.tolist()))
    diff = e0 ^ e1
    # every disagreement lies within the shell |d - R| < 2T ln(2^53) that
    # the coin's range allows, and there are few of them
    shell = 2 * T * math.log(TWO53) + 1e-9
    for (i, j) in diff:
        dth = abs(t[i] - t[j])
        dth = min(dth, 2 * math.pi - dth)
        d = math.acosh(math.cosh(r[i] - r[j]) + 2 * math.sinh(r[i]) * math.sinh(r[j]) * math.sin(dth / 2) ** 2)
        assert abs(d - R) < shell, (i, j, d, R)
    assert len(diff) < 0.02 * len(e0)
    assert len(e0) > 0.9 * n * k


def test_edge_frequency_follows_the_connection_probability():
    n = 3000
    a, R = O.solve_R(n, 8.0, 2.5)
    r, t, _ = O.sample(11, a, R, n)
    T = 0.5
    rp, col, _, ties = O.temp_csr(r, t, R, T, 11)
    assert ties == 0
    i, j, d = _distances(r, t)
    p = 1.0 / (1.0 + np.exp(np.clip((d - R) / (2 * T), -700, 700)))
    adj = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(rp))
    adj[rows, col] = True
    assert (adj == adj.T).all()
    hit = adj[i, j]
    # bins of p; per bin the edge count is a sum of independent Bernoulli(p)
    keep = p > 1e-5
    edges_q = np.quantile(p[keep], np.linspace(0, 1, 21))
    for lo, hi in zip(edges_q[:-1], edges_q[1:]):
        sel = keep & (p >= lo) & (p <= hi)
        mu = p[sel].sum()
        var = (p[sel] * (1 - p[sel])).sum()
        z = (hit[sel].sum() - mu) / math.sqrt(var)
        assert abs(z) < 5.0, (lo, hi, z)
    # the far pairs (p <= 1e-5) give at most a handful of edges
    far = ~keep
    assert hit[far].sum() <= p[far].sum() + 6 * math.sqrt(p[far].sum()) + 3


def test_mean_degree_matches_integration_of_the_model():
    n, k, g = 3000, 6.0, 3.0
    a, R = O.solve_R(n, k, g)
    T = 0.5
    exp_deg = expected_degree_temperature(n, a, R, T)
    means = []
    for seed in range(1, 9):
        r, t, _ = O.sample(seed, a, R, n)
        rp, _, _, ties = O.temp_csr(r, t, R, T, seed)
        assert ties == 0
        means.append(rp[-1] / n)
    means = np.array(means)
    se = means.std(ddof=1) / math.sqrt(len(means))
    assert abs(means.mean() - exp_deg) < 4 * se + 1e-9, (means, exp_deg)
    # and the temperature raises the degree above the threshold model's
    assert exp_deg > 1.3 * k


def test_coins_are_symmetric_and_uniform():
    rng = np.random.default_rng(3)
    pairs = rng.integers(0, 1 << 31, size=(4000, 2))
    us = []
    for i, j in pairs:
        if i == j:
            continue
        a = O.temp_coin(99, int(i), int(j))
        assert a == O.temp_coin(99, int(j), int(i))
        assert 1 <= a <= TWO53
        us.append(a / TWO53)
    assert stats.kstest(us, "uniform").pvalue > 1e-4
    # a different seed gives different coins
    assert O.temp_coin(98, 5, 9) != O.temp_coin(99, 5, 9)
    # coins of neighbouring pairs are unrelated
    row = [O.temp_coin(1, 0, j) / TWO53 for j in range(1, 3001)]
    assert abs(stats.pearsonr(row[:-1], row[1:])[0]) < 0.08
