"""Near-threshold point sets for the exactness tests of the search (test
infrastructure, CPU only).

Each constructed pair of points lies at a relative distance of about 2^-k
from the edge threshold cosh d = cosh R, on one side or the other, in a
regime where a fast search could go wrong:

* ``pi``: opposite points (dtheta near pi) with r1 + r2 near R, where the
  FP32 screen runs its full sine polynomial at its largest argument;
* ``mid``: angles between 2^-5 and 2.5 rad (the full polynomial, inner
  points);
* ``rim``: both points near the rim at angles of 1e-9 .. 1e-5 rad (the
  screen's two-term branch);
* ``edge``: the partner exactly on a radial band's inner edge, at the angle
  where the query window computed from that edge ends (times 1 -/+ 2^-k);
* ``cell``: the same with the partner on an angular cell boundary of many
  cell counts at once (angles c * 2 pi / 2^12);
* ``seam``: pairs straddling the 0 / 2 pi seam at the window's end;
* ``tie``: exact ties (the origin against the rim point r = R: distance R
  exactly), duplicates and near-duplicates.

The second point's radius (or angle) is solved in 60-digit arithmetic
(mpmath) from the distance law cosh d = cosh(r1 - r2) + 2 sinh r1 sinh r2
sin^2(dtheta/2) (native representation, Sec. 2.1) and then rounded to
binary64, so the final offsets are those of the rounded points; the oracle
decides every pair anyway.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

TWO_PI_D = 6.283185307179586
KS = (12, 14, 16, 17, 18, 19, 20, 22, 24, 28, 32, 36, 40, 44)
mp.mp.dps = 60


def coshd(r1, t1, r2, t2):
    """cosh of the hyperbolic distance of two binary64 points, 60 digits."""
    a, b = mp.mpf(t1), mp.mpf(t2)
    dt = abs(a - b)
    if dt > mp.pi:
        dt = 2 * mp.pi - dt
    s = mp.sin(dt / 2)
    r1, r2 = mp.mpf(r1), mp.mpf(r2)
    return mp.cosh(r1 - r2) + 2 * mp.sinh(r1) * mp.sinh(r2) * s * s


def rel_offset(R, r1, t1, r2, t2):
    """(cosh d - cosh R) / cosh R of the binary64 pair, as a float."""
    c = mp.cosh(mp.mpf(R))
    return float((coshd(r1, t1, r2, t2) - c) / c)


def _solve_r2(R, r1, t1, t2, eps, lo):
    """r2 in [lo, R] with cosh d = cosh R (1 + eps), or None."""
    target = mp.cosh(mp.mpf(R)) * (1 + mp.mpf(eps))
    f = lambda x: coshd(r1, t1, x, t2) - target  # noqa: E731
    a, b = mp.mpf(lo), mp.mpf(R)
    fa, fb = f(a), f(b)
    if fa * fb > 0:
        return None
    for _ in range(200):  # bisection: f increases on [lo, R] for our choices
        m = (a + b) / 2
        fm = f(m)
        if (fm > 0) == (fb > 0):
            b, fb = m, fm
        else:
            a, fa = m, fm
        if b - a < mp.mpf(2) ** -120:
            break
    r2 = float((a + b) / 2)
    return min(max(r2, 0.0), R)


def theta_max(R, r1, r2):
    """Angle at which the pair (r1, r2) is exactly at distance R (60 digits)."""
    r1, r2, R = mp.mpf(r1), mp.mpf(r2), mp.mpf(R)
    c = (mp.cosh(r1) * mp.cosh(r2) - mp.cosh(R)) / (mp.sinh(r1) * mp.sinh(r2))
    c = max(min(c, mp.mpf(1)), mp.mpf(-1))
    return mp.acos(c)


def _wrap(t):
    t = float(t) % TWO_PI_D
    return 0.0 if t >= TWO_PI_D else t


@functools.lru_cache(maxsize=8)
def constructed_pairs(R: float, edges: tuple, seed: int = 0):
    """List of (kind, k, side, r1, t1, r2, t2); side -1 aims inside, +1 outside."""
    rng = np.random.default_rng(seed)
    out = []

    def add(kind, k, side, r1, t1, r2, t2):
        if r2 is None or not (0.0 <= r1 <= R and 0.0 <= r2 <= R):
            return
        t1, t2 = _wrap(t1), _wrap(t2)
        out.append((kind, k, side, float(r1), t1, float(r2), t2))

    for k in KS:
        for side in (-1, 1):
            eps = side * 2.0 ** -k
            # opposite points, r1 + r2 near R
            for a in (-0.3 * R, 0.0, 0.2 * R):
                for d in (0.0, 1e-9, 1e-4, 0.1):
                    t1 = rng.uniform(0, TWO_PI_D)
                    t2 = _wrap(t1 + np.pi - d)
                    r1 = R / 2 + a
                    add("pi", k, side, r1, t1, _solve_r2(R, r1, t1, t2, eps, 0.0), t2)
            # middle angles, inner and middle radii
            for dth in (0.04, 0.2, 0.7, 1.5, 2.5):
                t1 = rng.uniform(0, TWO_PI_D)
                t2 = _wrap(t1 + dth)
                r1 = R * rng.uniform(0.35, 0.6)
                add("mid", k, side, r1, t1, _solve_r2(R, r1, t1, t2, eps, r1), t2)
            # rim pairs at small angles (the two-term sine branch)
            for r1 in (R - 1.5, R - 0.4, R - 1e-9):
                for r2t in (R - 1.0, R - 0.1, R):
                    r2t = max(r2t, r1)
                    ang = 2.0 * np.exp((R - r1 - r2t) / 2.0)
                    if not (ang < 2.0 ** -6):
                        continue
                    t1 = rng.uniform(0, TWO_PI_D)
                    t2 = _wrap(t1 + ang)
                    add("rim", k, side, r1, t1, _solve_r2(R, r1, t1, t2, eps, r1), t2)
    # the partner on a band's inner edge, at the window's end
    for E in edges[1:-1]:
        if E <= 0.25:
            continue
        for r1 in (R - E + 0.05, R - E + 1.0, R - 0.3, R):
            if not (0.0 < r1 <= R) or r1 + E <= R:
                continue
            th = theta_max(R, r1, E)
            for k in (8, 12, 16, 18, 20, 24, 28):
                for side in (-1, 1):
                    ang = th * (1 + side * mp.mpf(2) ** -k)
                    if ang >= mp.pi:
                        continue
                    t1 = rng.uniform(0, TWO_PI_D)
                    add("edge", k, side, r1, t1, E, t1 + float(ang))
                    # the partner on a cell boundary of every cell count up to 2^12
                    tb = TWO_PI_D * int(rng.integers(1, 4096)) / 4096.0
                    add("cell", k, side, r1, tb - float(ang), E, tb)
                    add("cell", k, side, r1, tb + float(ang), E, tb)
                    # across the seam
                    t1s = float(rng.choice([1e-12, 1e-7, 3e-4])) * float(min(th, 1.0))
                    add("seam", k, side, r1, t1s, E, TWO_PI_D + t1s - float(ang))
    # exact ties and duplicates
    for t in (0.0, 1.0, 3.0, TWO_PI_D - 1e-9):
        add("tie", 0, 0, 0.0, t, R, rng.uniform(0, TWO_PI_D))
        add("tie", 0, 0, 0.0, t, R, t)
        add("tie", 0, 0, 0.0, t, float(np.nextafter(R, 0.0)), t + 1.0)
        rr = R * rng.uniform(0.2, 1.0)
        add("tie", 0, 0, rr, t, rr, t)
        add("tie", 0, 0, rr, t, float(np.nextafter(rr, 0.0)), float(np.nextafter(t, 1.0)))
    return out


def point_set(R: float, alpha: float, edges, n_background: int, seed: int = 0):
    """Background points of the model's radial law (Eq. (1)) plus every
    constructed pair, shuffled; returns (r, theta, pairs, pair_index) where
    pair_index[p] gives the positions of pair p's two points."""
    rng = np.random.default_rng(1000 + seed)
    pairs = constructed_pairs(float(R), tuple(float(e) for e in edges), seed)
    u = rng.random(n_background)
    rb = np.arccosh(1.0 + u * (np.cosh(alpha * R) - 1.0)) / alpha
    rb = np.minimum(rb, R)
    tb = rng.uniform(0.0, TWO_PI_D, n_background)
    rp = np.array([[p[3], p[5]] for p in pairs], dtype=np.float64).ravel()
    tp = np.array([[p[4], p[6]] for p in pairs], dtype=np.float64).ravel()
    r = np.concatenate([rb, rp])
    t = np.concatenate([tb, tp])
    perm = rng.permutation(r.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    base = n_background + 2 * np.arange(len(pairs))
    pair_index = np.stack([inv[base], inv[base + 1]], axis=1)
    return r[perm].copy(), t[perm].copy(), pairs, pair_index
