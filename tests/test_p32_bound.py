"""The FP32 screen's error bound, pinned by emulation (CPU).

The search decides a pair from FP32 values when the normalised sum
    L = e'_q m'_c + m'_q e'_c + s'_q s'_c sin^2(dtheta/2)   (= cosh d / cosh R)
lies outside 1 -/+ 2^-18.  The design derives, with u = 2^-24, a relative
error of at most 21 u for L where the degree-11 sine polynomial runs (the
five Horner FMAs with rounded coefficients and a rounded x^2 at x = pi/2
contribute 4.7 u, the truncation 0.96 u) and at most 12 u on the two-term
branch (half-angle below 2^-6).  These tests emulate the kernel's exact
FP32 operation sequence (numpy float32; an FMA as the exact product plus
the addend in 64-bit-mantissa arithmetic, rounded once to float32) and
check the observed errors, on the arguments where they are largest,
against the derived bounds of each part: a dropped term in the derivation
(for example the Horner roundings, which the first statement of the bound
left out) shows up as an observed error above it."""
import numpy as np

U = 2.0 ** -24
F = np.float32
LD = np.longdouble
C5, C4, C3, C2, C1 = F(-1.0 / 39916800.0), F(1.0 / 362880.0), F(-1.0 / 5040.0), F(1.0 / 120.0), F(-1.0 / 6.0)


def fma32(a, b, c):
    return (np.asarray(a, F).astype(LD) * np.asarray(b, F).astype(LD) + np.asarray(c, F).astype(LD)).astype(F)


def sine_full(x):
    x = np.asarray(x, F)
    x2 = (x * x).astype(F)
    p = np.full_like(x, C5)
    for c in (C4, C3, C2, C1, F(1.0)):
        p = fma32(p, x2, c)
    return (x * p).astype(F)


def sine_short(x):
    x = np.asarray(x, F)
    x2 = (x * x).astype(F)
    return (x * fma32(x2, C1, F(1.0))).astype(F)


def test_longdouble_is_wide_enough():
    assert np.finfo(LD).nmant >= 63


def test_sine_square_full_polynomial():
    """(fl(s*s) - sin^2 X) / sin^2 X <= 2 sigma + u with sigma = 7.63 u:
    x rounding u, Horner 4.67 u, truncation 0.955 u, product u."""
    rng = np.random.default_rng(0)
    X = np.concatenate([np.pi / 2 - rng.random(400_000) * 1e-3, rng.random(400_000) * (np.pi / 2),
                        np.pi / 2 - rng.random(200_000) * 0.3]).astype(np.float64)
    s = sine_full(X.astype(F))
    s2 = (s * s).astype(F).astype(LD)
    ref = np.sin(X.astype(LD)) ** 2
    err = np.max(np.abs(s2 - ref) / ref) / U
    assert err <= 2 * 7.63 + 1.0 + 0.01, err
    # the bound is not loose by a factor: the worst case sits near pi / 2
    assert err > 4.0, err


def test_sine_square_short_branch():
    """Half-angle below 2^-6: sigma <= 3.01 u."""
    rng = np.random.default_rng(1)
    X = np.concatenate([rng.random(500_000) * 2.0 ** -6, np.exp(rng.uniform(np.log(1e-20), np.log(2.0 ** -6), 500_000))])
    s = sine_short(X.astype(F))
    s2 = (s * s).astype(F).astype(LD)
    ref = np.sin(X.astype(LD)) ** 2
    normal = ref >= LD(2.0 ** -126)
    err = np.max(np.abs(s2 - ref)[normal] / ref[normal]) / U
    assert err <= 2 * 3.01 + 1.0 + 0.01, err
    # below the normal range the square underflows: an absolute error of at
    # most half a subnormal step (plus the relative part), which the screen
    # counts as its absolute underflow term
    assert np.max(np.abs(s2 - ref)[~normal]) <= 2.0 ** -149


def _records(r, C):
    """The gather's FP32 record: binary64 values rounded once."""
    inv, sc = 1.0 / np.sqrt(2.0 * C), np.sqrt(2.0 / C)
    return (np.exp(r) * inv).astype(F), (np.exp(-r) * inv).astype(F), (np.sinh(r) * sc).astype(F)


def _screen_error(R, rq, rc, dth, full):
    C = np.cosh(R)
    eq, mq, sq = _records(rq, C)
    ec, mc, scc = _records(rc, C)
    x = (0.5 * dth).astype(F)
    s = sine_full(x) if full else sine_short(x)
    L = fma32(eq, mc, (mq * ec).astype(F))
    L = fma32((sq * scc).astype(F), (s * s).astype(F), L).astype(LD)
    rqL, rcL, dL = rq.astype(LD), rc.astype(LD), dth.astype(LD)
    ref = (np.cosh(rqL - rcL) + 2 * np.sinh(rqL) * np.sinh(rcL) * np.sin(dL / 2) ** 2) / LD(C)
    return np.max(np.abs(L - ref) / ref) / U


def test_screen_full_polynomial_near_threshold():
    """Inner pairs near the threshold with dtheta up to pi: at most 21 u."""
    rng = np.random.default_rng(2)
    worst = 0.0
    for R in (16.705267886314783, 25.670852, 36.91886526071599, 79.0):
        k = 200_000
        dth = np.concatenate([np.pi - rng.random(k) * 1e-3, rng.uniform(2.0 ** -5, np.pi, k)])
        rq = rng.uniform(0.0, R, 2 * k)
        # rc such that the pair is near the threshold for the larger angles
        rc = np.clip(R - rq + rng.normal(0.0, 0.05, 2 * k), 0.0, R)
        worst = max(worst, _screen_error(R, rq, rc, dth, True))
    assert worst <= 21.0, worst


def test_screen_short_branch_near_threshold():
    """Rim pairs at small angles near the threshold: at most 12 u."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for R in (16.705267886314783, 36.91886526071599, 79.0):
        k = 300_000
        rq = R - rng.random(k) * 3.0
        rc = R - rng.random(k) * 3.0
        dth = np.minimum(2.0 * np.exp((R - rq - rc) / 2.0) * rng.uniform(0.5, 1.5, k), 2.0 ** -5)
        worst = max(worst, _screen_error(R, rq, rc, dth, False))
    assert worst <= 12.0, worst


def test_band_covers_bound():
    """The accept/reject band 2^-18 = 64 u exceeds both bounds with margin."""
    assert 2.0 ** -18 / U == 64.0
    assert 21.0 * 3 <= 64.0 and 12.0 * 5 <= 64.0
