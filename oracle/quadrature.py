"""Quadrature rules on the reference triangle and interval (oracle).

Sec. 3 (spatial discretisation) integrates regular panel integrals with Gaussian
rules and weakly singular ones after a Duffy transformation, without naming
orders.  Reading used here:
  * regular integrals: the classical 7-point rule of degree 5 (Radon; tabulated
    by Strang-Fix and Dunavant) -- centroid plus two orbits of three points;
  * near-singular panels: the same rule on the 16 sub-triangles of two levels of
    midpoint subdivision (112 points);
  * the remaining 1D integral of the self panel: 16-point Gauss-Legendre.
"""
from __future__ import annotations

import math

import numpy as np


def radon7():
    """Barycentric points (7, 3) and weights (7,) summing to 1."""
    sq = math.sqrt(15.0)
    a = (6.0 - sq) / 21.0
    b = (6.0 + sq) / 21.0
    wa = (155.0 - sq) / 1200.0
    wb = (155.0 + sq) / 1200.0
    pts = [(1 / 3, 1 / 3, 1 / 3),
           (a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a),
           (b, b, 1 - 2 * b), (b, 1 - 2 * b, b), (1 - 2 * b, b, b)]
    w = [9.0 / 40.0] + [wa] * 3 + [wb] * 3
    return np.array(pts, dtype=np.float64), np.array(w, dtype=np.float64)


def gauss_legendre01(n: int):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def subdivide(v0, v1, v2, levels: int):
    """Midpoint (4-fold) subdivision of a triangle, ``levels`` times.  Returns a
    list of (a, b, c) vertex triples, all with the orientation of the parent."""
    tris = [(np.asarray(v0, float), np.asarray(v1, float), np.asarray(v2, float))]
    for _ in range(levels):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = nxt
    return tris


def triangle_rule(v0, v1, v2, levels: int = 0):
    """Points (q, 3) and weights (q,) -- weights include the area -- of the
    7-point rule applied on each sub-triangle of ``levels`` midpoint
    subdivisions of the triangle (v0, v1, v2)."""
    bary, w = radon7()
    P, W = [], []
    for a, b, c in subdivide(v0, v1, v2, levels):
        area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
        P.append(bary[:, 0:1] * a + bary[:, 1:2] * b + bary[:, 2:3] * c)
        W.append(w * area)
    return np.concatenate(P), np.concatenate(W)
