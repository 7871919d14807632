"""Pins for the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms from the paper (Eq. (1), Eq. (2), Eq. (3),
Proposition 1, Lemmas 1 and 2, gamma = 2 alpha + 1), an independent numerical
integration of the model's expected degree, or a 100-digit evaluation of the
Poincare metric.  These run on the CPU (no GPU).
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

import oracle as O
from quadrature import expected_degree

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (n, target average degree, gamma)
C1 = (10_000, 6.0, 3.0)
C2 = (1_000_000, 10.0, 2.7)
C3 = (100_000_000, 20.0, 2.2)
C5_LARGE = (10_000_000, 16.0, 2.5)
TWO_PI_D = 6.283185307179586


def setup_module(_):
    O.build(force=False)


# ---------------------------------------------------------------- RNG ----

def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for w in rows:
        v = [int(x, 16) for x in w]
        got = O.philox4x32_10(v[0:4], v[4:6]).tolist()
        assert got == v[6:10]


def test_uniform_words_and_theta_product():
    seed = 0x0123456789ABCDEF
    for i in [0, 1, 7, 2**32 - 1, 2**32, 123456789012]:
        ctr = [i & 0xFFFFFFFF, i >> 32, 0, 0]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        x = [int(v) for v in O.philox4x32_10(ctr, key)]
        ut, ur = O.uniforms(seed, i)
        assert ut == (((x[1] << 32) | x[0]) >> 11) * 2.0**-53
        assert ur == (((x[3] << 32) | x[2]) >> 11) * 2.0**-53
    a, R = O.solve_R(*C1)
    r, t, _ = O.sample(seed, a, R, 64, i0=1000)
    for k in range(64):
        ut, _ = O.uniforms(seed, 1000 + k)
        assert t[k] == np.float64(TWO_PI_D) * np.float64(ut)
        assert 0.0 <= t[k] < 2 * math.pi


# ------------------------------------------------------------ radius R ----

@pytest.mark.parametrize("cfg", [C1, C2, C3, C5_LARGE])
def test_R_gives_target_degree_by_exact_integration(cfg):
    """Eq. (22) read with (pi-1)*zeta/alpha, zeta = 1: the exact expected
    degree at the solved R is the target to within 0.1 %."""
    n, k, g = cfg
    a, R = O.solve_R(n, k, g)
    assert a == (g - 1.0) * 0.5
    e = expected_degree(n, a, R)
    assert abs(e / k - 1.0) < 1e-3, (R, e)


def test_R_is_the_first_double_at_or_below_target():
    for n, k, g in [C1, C2, C3, C5_LARGE, (1000, 64.0, 2.1), (10**6, 4.0, 3.5)]:
        a, R = O.solve_R(n, k, g)
        assert O.kbar_minus(n, a, R, k) <= 0.0
        assert O.kbar_minus(n, a, np.nextafter(R, 0.0), k) > 0.0


def test_eq22_literal_xi_reading_is_rejected():
    """The printed '(pi-1) xi/alpha' term: for heavy tails (gamma 2.1-2.2) it
    never reaches the target, and where it does cross the target the exact
    expected degree there misses the target by far more than the corrected
    reading does."""
    for n, k, g in [C3, (1000, 64.0, 2.1)]:
        a = O.alpha(g)
        Rs = np.linspace(0.5, 2 * math.log(n) + 40, 3000)
        assert max(O.kbar_eq22(n, a, R, literal=True) for R in Rs) < k
    for n, k, g in [C2, C5_LARGE]:
        a, R = O.solve_R(n, k, g)
        exact_err = abs(expected_degree(n, a, R) / k - 1.0)
        lit_err = abs(O.kbar_eq22(n, a, R, literal=True) / k - 1.0)
        assert lit_err > 0.002 and lit_err > 10 * exact_err


def test_eq22_decreasing_past_its_peak_over_batch_ranges():
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(round(10 ** (3 + 3 * rng.random())))
        k = 4 + 60 * rng.random()
        g = 2.1 + 1.4 * rng.random()
        a, R = O.solve_R(n, k, g)
        grid = np.linspace(R - 0.5 * R, 2 * math.log(n) + 40, 400)
        vals = np.array([O.kbar_eq22(n, a, x) for x in grid])
        peak = int(np.argmax(vals))
        assert np.all(np.diff(vals[peak:]) < 0)
        e = expected_degree(n, a, R, panels=24, nodes=16)
        # Eq. (22) is asymptotic: it undershoots at small n, never overshoots
        assert -0.11 < e / k - 1.0 < 2e-3


# ---------------------------------------------------------------- points ----

def _F(r, a, R):
    return (np.cosh(a * r) - 1.0) / (np.cosh(a * R) - 1.0)


@pytest.mark.parametrize("cfg", [C1, C3])
def test_radius_and_angle_distributions_ks(cfg):
    n, k, g = cfg
    a, R = O.solve_R(n, k, g)
    r, t, hard = O.sample(9, a, R, 200_000)
    assert hard == 0
    assert r.min() >= 0.0 and r.max() <= R
    assert stats.kstest(_F(r, a, R), "uniform").pvalue > 1e-3
    assert stats.kstest(t / (2 * math.pi), "uniform").pvalue > 1e-3


def test_radius_is_correctly_rounded():
    """r = acosh(1 + u (cosh(alpha R) - 1)) / alpha (inverse of the CDF in
    Appendix C) rounded to nearest, checked against 60-digit mpmath."""
    mp.mp.dps = 60
    rng = np.random.default_rng(5)
    for n, k, g in [C1, C3, (1000, 64.0, 2.1)]:
        a, R = O.solve_R(n, k, g)
        us = list(rng.random(150)) + [0.0, 2.0**-53, 2.0**-40, 1e-9, 0.5, 1 - 2.0**-53, 1 - 1e-12]
        for u in us:
            u = float(np.floor(u * 2**53) / 2**53)
            c = mp.cosh(mp.mpf(a) * mp.mpf(R)) - 1
            x = mp.mpf(u) * c
            ref = mp.log1p(x + mp.sqrt(x * (x + 2))) / mp.mpf(a)
            got, hard = O.radius(u, a, R)
            assert not hard
            assert got == float(ref), (u, got, float(ref))


def _split_radius(a, lo, hi):
    """Eq. (3): the radius that halves the probability mass of [lo, hi)."""
    return math.acosh((math.cosh(a * hi) + math.cosh(a * lo)) / 2.0) / a


def _quadtree_cells(a, R, depth):
    cells = [(0.0, 2 * math.pi, 0.0, R)]
    for _ in range(depth):
        nxt = []
        for (p0, p1, r0, r1) in cells:
            pm = 0.5 * (p0 + p1)
            rm = _split_radius(a, r0, r1)
            nxt += [(p0, pm, r0, rm), (pm, p1, r0, rm), (p0, pm, rm, r1), (pm, p1, rm, r1)]
        cells = nxt
    return cells


def test_lemma1_cells_at_depth_k_are_equiprobable():
    a, R = O.solve_R(*C3)
    depth = 3
    r, t, _ = O.sample(21, a, R, 100_000)
    cells = _quadtree_cells(a, R, depth)
    counts = np.zeros(len(cells))
    for ci, (p0, p1, r0, r1) in enumerate(cells):
        counts[ci] = np.count_nonzero((t >= p0) & (t < p1) & (r >= r0) & (r < r1))
    counts[-1] += np.count_nonzero(r >= R)  # r may round up to R itself
    assert counts.sum() == r.size
    chi = stats.chisquare(counts)
    assert chi.pvalue > 1e-3


def test_lemma2_max_load_on_complete_tree():
    """With k = ceil(log4 n), no equal-probability leaf holds more than
    3 ln n / ln ln n points (balls into bins)."""
    n = 4**8
    a, R = O.solve_R(n, 8.0, 2.5)
    r, t, _ = O.sample(3, a, R, n)
    k = math.ceil(math.log(n, 4))
    side = 2**k
    # equal-mass radial boundaries of the complete tree (Eq. (3) applied k
    # times gives the CDF quantiles j / 2^k)
    ri = np.minimum((_F(r, a, R) * side).astype(np.int64), side - 1)
    ti = np.minimum((t / (2 * math.pi) * side).astype(np.int64), side - 1)
    load = np.bincount(ri * side + ti, minlength=side * side)
    assert load.max() <= 3 * math.log(n) / math.log(math.log(n))


def test_eq3_split_matches_cdf_median():
    a, R = O.solve_R(*C2)
    for lo, hi in [(0.0, R), (3.0, 9.0), (R - 1, R)]:
        m = _split_radius(a, lo, hi)
        assert _F(m, a, R) - _F(lo, a, R) == pytest.approx(_F(hi, a, R) - _F(m, a, R), rel=1e-9)


# ------------------------------------------------------- edge relation ----

def _mp_dist_poincare(r1, t1, r2, t2):
    """Eq. (2) on the points mapped by mapToPoincare (Appendix B.2)."""
    def to_disk(r, t):
        rr = mp.sqrt((mp.cosh(r) - 1) / (mp.cosh(r) + 1))
        return rr * mp.cos(t), rr * mp.sin(t), rr
    x1, y1, n1 = to_disk(mp.mpf(r1), mp.mpf(t1))
    x2, y2, n2 = to_disk(mp.mpf(r2), mp.mpf(t2))
    d2 = (x1 - x2) ** 2 + (y1 - y2) ** 2
    return mp.acosh(1 + 2 * d2 / ((1 - n1**2) * (1 - n2**2)))


def _mp_theta_max(r1, r2, R):
    r1, r2, R = mp.mpf(r1), mp.mpf(r2), mp.mpf(R)
    s2 = (mp.cosh(R) - mp.cosh(r1 - r2)) / (2 * mp.sinh(r1) * mp.sinh(r2))
    return 2 * mp.asin(mp.sqrt(s2))


def _near_threshold_pairs(R, rng, count, rim):
    out = []
    while len(out) < count:
        if rim:
            r1 = R - 3 * rng.random()
            r2 = R - 3 * rng.random()
        else:
            r1 = R * rng.random()
            r2 = R * rng.random()
        if r1 + r2 <= R * 1.0001:
            continue
        tm = _mp_theta_max(r1, r2, R)
        k = rng.integers(3, 14)
        sgn = 1 if rng.random() < 0.5 else -1
        dth = float(tm * (1 + sgn * mp.mpf(10) ** (-int(k))))
        t1 = 2 * math.pi * rng.random()
        t2 = t1 + dth
        if t2 >= TWO_PI_D:
            t2 -= TWO_PI_D
        if not (0 <= t2 < TWO_PI_D):
            continue
        out.append((r1, t1, r2, t2))
    return out


@pytest.mark.parametrize("cfg,rim", [(C1, True), (C3, True), (C3, False), (C2, False)])
def test_edge_decision_equals_poincare_metric_near_threshold(cfg, rim):
    mp.mp.dps = 100
    a, R = O.solve_R(*cfg)
    rng = np.random.default_rng(17)
    for (r1, t1, r2, t2) in _near_threshold_pairs(R, rng, 120, rim):
        ref = _mp_dist_poincare(r1, t1, r2, t2) <= mp.mpf(R)
        e, _, ties = O.is_edge(r1, t1, r2, t2, R)
        assert ties == 0
        assert e == ref, (r1, t1, r2, t2)
        assert O.is_edge(r2, t2, r1, t1, R)[0] == e


def test_literal_distance_law_loses_rim_decisions_that_the_oracle_keeps():
    """Why the oracle decides on the rewritten (non-negative sum) form: the
    printed law evaluated literally in binary64 cancels two products of
    about e^{2r}/4 down to cosh R, so its error grows like e^R ulp.  On rim
    pairs placed 1e-3 .. 1e-14 (relative) from the threshold it gets a
    growing share wrong as R grows, while the oracle's decision matches
    100-digit arithmetic on every pair at every radius."""
    mp.mp.dps = 100
    wrong = {}
    for name, cfg in (("C1", C1), ("C3", C3)):
        a, R = O.solve_R(*cfg)
        rng = np.random.default_rng(29)
        wrong_lit = wrong_orc = total = 0
        for (r1, t1, r2, t2) in _near_threshold_pairs(R, rng, 150, rim=True):
            ref = _mp_dist_poincare(r1, t1, r2, t2) <= mp.mpf(R)
            wrong_orc += O.is_edge(r1, t1, r2, t2, R)[0] != ref
            wrong_lit += O.is_edge_literal(r1, t1, r2, t2, R) != ref
            total += 1
        assert wrong_orc == 0, name
        wrong[name] = wrong_lit
    assert wrong["C3"] >= 150 // 4 and wrong["C3"] > 1.5 * wrong["C1"], wrong


def test_edge_decision_equals_proposition1_circle():
    """Algorithm 1's range query: w is a neighbour of v iff w's Poincare image
    lies in the Euclidean circle of Proposition 1 around v's image."""
    mp.mp.dps = 100
    a, R = O.solve_R(*C2)
    rng = np.random.default_rng(23)
    pairs = _near_threshold_pairs(R, rng, 80, rim=False)
    for (r1, t1, r2, t2) in pairs:
        rh = mp.sqrt((mp.cosh(r1) - 1) / (mp.cosh(r1) + 1))
        A = mp.cosh(mp.mpf(R)) - 1
        B = 1 - rh**2
        cen = 2 * rh / (A * B + 2)
        rad = mp.sqrt(cen**2 - (2 * rh**2 - A * B) / (A * B + 2))
        cx, cy = cen * mp.cos(t1), cen * mp.sin(t1)
        rw = mp.sqrt((mp.cosh(r2) - 1) / (mp.cosh(r2) + 1))
        wx, wy = rw * mp.cos(t2), rw * mp.sin(t2)
        inside = (wx - cx) ** 2 + (wy - cy) ** 2 <= rad**2
        assert O.is_edge(r1, t1, r2, t2, R)[0] == inside


def test_edge_special_cases():
    a, R = O.solve_R(*C3)
    rng = np.random.default_rng(3)
    for _ in range(200):
        rj, tj, ti = R * rng.random(), TWO_PI_D * rng.random(), TWO_PI_D * rng.random()
        # a vertex at the origin is at distance r_j from every other vertex
        assert O.is_edge(0.0, ti, rj, tj, R)[0]
        assert O.is_edge(0.0, ti, R, tj, R)[0]
        # equal angles: distance |r_i - r_j| <= R
        ri = R * rng.random()
        assert O.is_edge(ri, tj, rj, tj, R)[0]
        # the same point twice
        assert O.is_edge(ri, ti, ri, ti, R)[0]
    # opposite angles: distance r_i + r_j (up to the rounding of pi)
    for eps in [1e-6, 1e-9, 1e-12]:
        ri = 0.4 * R
        rj_in = R * (1 - eps) - ri
        rj_out = R * (1 + eps) - ri
        assert O.is_edge(ri, 0.0, rj_in, math.pi, R)[0]
        assert not O.is_edge(ri, 0.0, rj_out, math.pi, R)[0]


def test_wraparound_pairs():
    mp.mp.dps = 100
    a, R = O.solve_R(*C3)
    rng = np.random.default_rng(8)
    for _ in range(60):
        r1, r2 = R - rng.random(), R - rng.random()
        tm = float(_mp_theta_max(r1, r2, R))
        t1 = tm * rng.random()
        t2 = TWO_PI_D - (tm - t1) * (1 + (rng.random() - 0.5) * 1e-6)
        ref = _mp_dist_poincare(r1, t1, r2, t2) <= mp.mpf(R)
        assert O.is_edge(r1, t1, r2, t2, R)[0] == ref


def test_binary64_screen_agrees_with_binary128():
    a, R = O.solve_R(*C1)
    rng = np.random.default_rng(4)
    r, t, _ = O.sample(77, a, R, 3000)
    quad_calls = 0
    for _ in range(6000):
        i, j = rng.integers(0, 3000, 2)
        if i == j:
            continue
        e, q, ties = O.is_edge(r[i], t[i], r[j], t[j], R)
        quad_calls += q
        assert e == O.is_edge_quad(r[i], t[i], r[j], t[j], R)
        assert ties == 0
    for (r1, t1, r2, t2) in _near_threshold_pairs(R, rng, 100, rim=True):
        assert O.is_edge(r1, t1, r2, t2, R)[0] == O.is_edge_quad(r1, t1, r2, t2, R)


# ------------------------------------------------------------- graphs ----

def test_bruteforce_graph_is_simple_and_symmetric():
    a, R, r, t, row_ptr, col, st = O.generate(*C1, seed=1)
    n = C1[0]
    assert st["ties"] == 0 and st["near_midpoint"] == 0
    assert row_ptr[-1] == col.size and col.size % 2 == 0
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    assert not np.any(src == col)
    fwd = src * n + col
    bwd = col.astype(np.int64) * n + src
    assert np.array_equal(np.sort(fwd), np.sort(bwd))
    for i in range(n):
        seg = col[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)
    # sampled rows agree with the full CSR
    which = np.array([0, 5, 77, 9999], dtype=np.int64)
    ptr, rc, _, _ = O.rows(r, t, R, which)
    for a_, i in enumerate(which):
        assert np.array_equal(rc[ptr[a_]:ptr[a_ + 1]], col[row_ptr[i]:row_ptr[i + 1]])


def test_mean_degree_matches_exact_expectation_over_seeds():
    n, k, g = C1
    a, R = O.solve_R(n, k, g)
    exp_deg = expected_degree(n, a, R)
    means = []
    for seed in range(1, 9):
        r, t, _ = O.sample(seed, a, R, n)
        deg, _, ties = O.degrees(r, t, R)
        assert ties == 0
        means.append(deg.mean())
    means = np.array(means)
    se = means.std(ddof=1) / math.sqrt(len(means))
    assert abs(means.mean() - exp_deg) < 4 * se + 1e-9, (means, exp_deg)


def test_degree_decays_as_exp_minus_r_over_2():
    """Expected degree at radius r falls as e^{-r/2}; with the radial density
    of Eq. (1) this gives the power-law exponent gamma = 2 alpha + 1 (Sec. 2.1)."""
    n, k, g = (20_000, 10.0, 2.6)
    a, R = O.solve_R(n, k, g)
    r, t, _ = O.sample(31, a, R, n)
    deg, _, _ = O.degrees(r, t, R)
    lo, hi = R / 2 + 1.0, R - 1.5
    edges = np.linspace(lo, hi, 9)
    xs, ys = [], []
    for b0, b1 in zip(edges[:-1], edges[1:]):
        m = (r >= b0) & (r < b1)
        if m.sum() > 30:
            xs.append(r[m].mean())
            ys.append(np.log(deg[m].mean()))
    slope = np.polyfit(xs, ys, 1)[0]
    assert abs(slope + 0.5) < 0.06, slope
    # the radial density of Eq. (1) carries alpha: its maximum-likelihood
    # estimate from the sample recovers alpha, hence gamma = 2 alpha + 1
    from scipy.optimize import minimize_scalar

    def nll(x):
        return -np.sum(np.log(x * np.sinh(x * r) / (np.cosh(x * R) - 1.0)))

    fit = minimize_scalar(nll, bounds=(0.51, 2.0), method="bounded")
    assert fit.x == pytest.approx(a, rel=0.02)
