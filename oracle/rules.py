"""Fully symmetric triangle rules of degree 2p and the prism rule built on them.

TEST INFRASTRUCTURE ONLY (part of the oracle): imported by ``tests/``, the
smoke check and the benchmark's CPU-baseline leg, never by the product.

The paper's Table 3 gives 4 N_I quadrature scalars per degree (24, 72, 192,
320, 600, 924, 1344 for p = 1..7), so N_I = 6, 18, 48, 80, 150, 231, 336 =
(3, 6, 12, 16, 25, 33, 42) x (p + 1).  Read here as a fully symmetric
triangle rule of degree 2p with that many points times the (p+1)-point
Gauss-Legendre rule in zeta; the paper states the accuracy requirement
(products of shape functions integrated exactly, Sec. 2) but names no rule.

A fully symmetric triangle rule is a union of orbits of the permutations of
the barycentric coordinates (lambda0, lambda1, lambda2): the centroid (one
point), 3-orbits (a, a, 1-2a) and 6-orbits (a, b, 1-a-b).  Its orbit weights
and parameters solve the moment equations

    sum_q w_q xi1^i xi2^j = i! j! / (i + j + 2)!      (i + j <= 2p)

on the reference triangle (area 1/2, xi1 = lambda1, xi2 = lambda2).  These
equations have several positive interior solutions for some degrees; the rule
taken is the one nearest the six-digit starting values below, solved by
Gauss-Newton in 40-digit arithmetic (mpmath) with exact rational right-hand
sides and rounded to double at the end.

Point order (the element tables of the GPU library follow the same
specification): centroid first, then each 3-orbit (listed order) as
(a, a, 1-2a), (a, 1-2a, a), (1-2a, a, a), then each 6-orbit with a < b < c =
1-a-b as (a,b,c), (a,c,b), (b,a,c), (b,c,a), (c,a,b), (c,b,a), all as
barycentric triples.  Prism point q = k * ntri + t (t triangle point, k
Gauss point in zeta, ascending), weight w_t * w_k.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import factorial

import mpmath as mp
import numpy as np

# Starting values per degree p: centroid weights, 3-orbits (w, a), 6-orbits
# (w, a, b).  Weights sum to the triangle area 1/2.
START = {
    1: ([], [(0.166667, 0.166667)], []),
    2: ([], [(0.0549759, 0.0915762), (0.111691, 0.445948)], []),
    3: ([], [(0.0254225, 0.0630890), (0.0583931, 0.249287)], [(0.0414255, 0.0531450, 0.310352)]),
    4: ([0.0721578], [(0.0162292, 0.0505472), (0.0516087, 0.170569), (0.0475458, 0.459293)],
        [(0.0136152, 0.00839478, 0.263113)]),
    5: ([0.0399473], [(0.00411191, 0.0233089), (0.0355619, 0.425086)],
        [(0.0186799, 0.0299460, 0.358740), (0.0154433, 0.0356326, 0.143295),
         (0.0227153, 0.147926, 0.223767)]),
    6: ([], [(0.00396582, 0.0246464), (0.0142430, 0.109258), (0.0312706, 0.271463),
             (0.0249592, 0.440112), (0.0121334, 0.488204)],
        [(0.00754184, 0.0213825, 0.127280), (0.0108918, 0.0230342, 0.291656),
         (0.0216137, 0.116296, 0.255454)]),
    7: ([], [(0.00246170, 0.0193910), (0.00721685, 0.0617999), (0.0210813, 0.177206),
             (0.0258871, 0.273478), (0.0163942, 0.417645), (0.0109418, 0.488964)],
        [(0.00250511, 0.00126833, 0.118974), (0.00721815, 0.0146470, 0.298373),
         (0.0123329, 0.0571248, 0.172267), (0.0192858, 0.0929162, 0.336861)]),
}

DPS = 40


def _points(theta, shape):
    """Barycentric points and weights of the orbits with parameters theta
    (flat: centroid weights, then (w, a) per 3-orbit, then (w, a, b) per 6-orbit)."""
    n0, n1, n2 = shape
    out = []
    i = 0
    for _ in range(n0):
        w = theta[i]; i += 1
        third = mp.mpf(1) / 3
        out.append((w, (third, third, third)))
    for _ in range(n1):
        w, a = theta[i], theta[i + 1]; i += 2
        c = 1 - 2 * a
        out += [(w, (a, a, c)), (w, (a, c, a)), (w, (c, a, a))]
    for _ in range(n2):
        w, a, b = theta[i], theta[i + 1], theta[i + 2]; i += 3
        c = 1 - a - b
        out += [(w, (a, b, c)), (w, (a, c, b)), (w, (b, a, c)), (w, (b, c, a)), (w, (c, a, b)), (w, (c, b, a))]
    return out


def _residual(theta, shape, deg):
    pts = _points(theta, shape)
    r = []
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            exact = Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
            s = mp.mpf(0)
            for w, lam in pts:
                s += w * lam[1] ** i * lam[2] ** j
            r.append(s - mp.mpf(exact.numerator) / exact.denominator)
    return mp.matrix(r)


@lru_cache(maxsize=None)
def triangle_rule(p: int):
    """(xi [ntri, 2], w [ntri]) of the symmetric triangle rule of degree 2p."""
    c0, s3, s6 = START[p]
    shape = (len(c0), len(s3), len(s6))
    with mp.workdps(DPS):
        theta = [mp.mpf(v) for v in c0] + [mp.mpf(v) for o in s3 for v in o] + [mp.mpf(v) for o in s6 for v in o]
        h = mp.mpf(10) ** (-DPS // 2)
        for _ in range(40):
            r = _residual(theta, shape, 2 * p)
            J = mp.matrix(len(r), len(theta))
            for k in range(len(theta)):                 # central differences
                tp = list(theta); tm = list(theta)
                tp[k] += h; tm[k] -= h
                col = (_residual(tp, shape, 2 * p) - _residual(tm, shape, 2 * p)) / (2 * h)
                for m in range(len(r)):
                    J[m, k] = col[m]
            step = mp.lu_solve(J.T * J, -(J.T * r))     # Gauss-Newton (consistent system)
            theta = [t + step[k] for k, t in enumerate(theta)]
            if mp.norm(step) < mp.mpf(10) ** (-DPS + 8):
                break
        else:
            raise RuntimeError(f"triangle rule p={p}: Gauss-Newton did not converge")
        pts = _points(theta, shape)
        xi = np.array([[float(lam[1]), float(lam[2])] for _, lam in pts])
        w = np.array([float(wt) for wt, _ in pts])
    return xi, w


def prism_rule(p: int, gauss_legendre):
    """(pts [nq, 3] = (xi1, xi2, zeta), w [nq]) of the symmetric triangle rule
    x (p+1)-point Gauss-Legendre in zeta; `gauss_legendre(n)` returns the
    oracle's nodes and weights on [-1, 1]."""
    xi, wt = triangle_rule(p)
    z, wz = gauss_legendre(p + 1)
    ntri = len(wt)
    pts = np.zeros(((p + 1) * ntri, 3))
    w = np.zeros((p + 1) * ntri)
    for k in range(p + 1):
        pts[k * ntri:(k + 1) * ntri, :2] = xi
        pts[k * ntri:(k + 1) * ntri, 2] = z[k]
        w[k * ntri:(k + 1) * ntri] = wt * wz[k]
    return pts, w
