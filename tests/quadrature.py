"""Expected average degree of the threshold RHG model by numerical integration.

Independent of Eq. (22): it integrates the model's definition directly.  A
vertex at radius r1 is joined to a vertex at radius r2 whenever their angle
difference is at most theta_max(r1, r2) (the angle at which the distance
reaches R), and the angle difference is uniform on [0, pi], so
    E[deg] = (n - 1) * int int f(r1) f(r2) theta_max(r1, r2)/pi dr1 dr2
with f the radial density of Eq. (1) and theta_max = pi when r1 + r2 <= R,
else 2 asin(sqrt((cosh R - cosh(r1 - r2)) / (2 sinh r1 sinh r2))).
"""
import math

import numpy as np


def _gl(a, b, m):
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def expected_degree(n, alpha, R, panels=48, nodes=24):
    cRm1 = np.expm1(alpha * R) / 2 + np.expm1(-alpha * R) / 2  # cosh(aR) - 1

    def f(r):
        return alpha * np.sinh(alpha * r) / cRm1

    def F(r):  # CDF of Eq. (1)
        return (np.cosh(alpha * r) - 1.0) / cRm1

    # outer nodes on a grid graded towards the rim, where the mass is
    edges = R * (1.0 - np.linspace(1.0, 0.0, panels + 1) ** 2)
    xs, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        x, w = _gl(a, b, nodes)
        xs.append(x)
        ws.append(w)
    r1 = np.concatenate(xs)
    w1 = np.concatenate(ws)
    # inner integral: r2 in [0, R - r1] contributes F(R - r1) (always joined);
    # r2 = (R - r1) + t^2, t in [0, sqrt(r1)] removes the square-root kink.
    t01, wt01 = np.polynomial.legendre.leggauss(4 * nodes)
    total = 0.0
    for r, w in zip(r1, w1):
        inner = F(R - r)
        tmax = np.sqrt(r)
        t = 0.5 * tmax * (t01 + 1.0)
        wt = 0.5 * tmax * wt01
        r2 = (R - r) + t * t
        s2 = (np.cosh(R) - np.cosh(r - r2)) / (2.0 * np.sinh(r) * np.sinh(r2))
        s2 = np.clip(s2, 0.0, 1.0)
        th = 2.0 * np.arcsin(np.sqrt(s2))
        inner += np.sum(wt * 2.0 * t * f(r2) * th / np.pi)
        total += w * f(r) * inner
    return (n - 1) * total


def expected_degree_temperature(n, alpha, R, T, panels=24, nodes=12, phi_panels=64, phi_nodes=8):
    """Expected average degree of the temperature model, integrated from its
    definition: a pair at radii (r1, r2) and angle difference phi (uniform on
    [0, pi]) is joined with probability p(d) = 1 / (1 + e^{(d - R)/(2T)}), so
        E[deg] = (n - 1) * int int f(r1) f(r2) (1/pi) int_0^pi p(d) dphi dr1 dr2.
    The angle is integrated in y = ln(phi) (d grows like 2 ln phi for small
    phi, so p is a logistic curve of width ~T in y), the radii on grids graded
    towards the rim."""
    cRm1 = np.expm1(alpha * R) / 2 + np.expm1(-alpha * R) / 2

    def f(r):
        return alpha * np.sinh(alpha * r) / cRm1

    edges = R * (1.0 - np.linspace(1.0, 0.0, panels + 1) ** 2)
    xs, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        x, w = _gl(a, b, nodes)
        xs.append(x)
        ws.append(w)
    r = np.concatenate(xs)
    wr = np.concatenate(ws) * f(r)
    ylo, yhi = math.log(1e-14), math.log(math.pi)
    yedges = np.linspace(ylo, yhi, phi_panels + 1)
    ys, wys = [], []
    for a, b in zip(yedges[:-1], yedges[1:]):
        x, w = _gl(a, b, phi_nodes)
        ys.append(x)
        wys.append(w)
    y = np.concatenate(ys)
    phi = np.exp(y)
    wphi = np.concatenate(wys) * phi / math.pi        # dphi = phi dy, uniform density 1/pi
    s2 = np.sin(0.5 * phi) ** 2
    total = 0.0
    for i in range(r.shape[0]):
        r1 = r[i]
        # cosh d = cosh(r1 - r2) + 2 sinh r1 sinh r2 sin^2(phi/2), all terms >= 0
        ch = np.cosh(r1 - r)[:, None] + 2.0 * np.sinh(r1) * np.sinh(r)[:, None] * s2[None, :]
        d = np.log(ch) + np.log1p(np.sqrt(1.0 - 1.0 / (ch * ch)))   # acosh without overflow of ch^2
        z = np.clip((d - R) / (2.0 * T), -700.0, 700.0)
        p = 1.0 / (1.0 + np.exp(z))
        inner = p @ wphi + 1e-14 / math.pi * p[:, 0]    # the sliver phi < 1e-14 at p(phi_min)
        total += wr[i] * float(inner @ wr)
    return (n - 1) * total
