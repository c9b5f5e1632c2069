"""Laplace-domain single-layer entries (oracle).

V(s)[i, j] = integral over tau_j of U(x_i - y, s) dy, with the Laplace transform
of the retarded fundamental solution (Sec. 2, eq. slp; Sec. 3, where every
kernel is replaced by its transform),

    U(r, s) = exp(-s r / c) / (4 pi r),   Re s > 0,

collocated at the centroid x_i of tau_i with piecewise-constant psi_j
(Sec. 3, semi-discrete collocation system).  The paper fixes neither the
collocation points for psi nor the quadrature orders; the reading used:

  self  (i == j)            Duffy-type split of tau_i at x_i into three
                            sub-triangles; the radial integral is done in
                            closed form and the remaining polar angle by
                            16-point Gauss-Legendre per sub-triangle.
  near  (|x_i - x_j| < 2 h_j) 7-point rule on 16 sub-triangles (112 points).
  far   (otherwise)           7-point rule.
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature
from .geometry import sqnorm

FOUR_PI = 4.0 * math.pi
SELF, NEAR, FAR = 0, 1, 2


def kernel(r, s, c):
    """U(r, s) = exp(-s r / c) / (4 pi r); broadcasts r against s."""
    return np.exp(-s * r / c) / (FOUR_PI * r)


def phi(a):
    """(1 - exp(-a)) / a, the exact value of int_0^1 exp(-a u) du; its Taylor
    series 1 - a/2 + a^2/6 - a^3/24 is used for |a| < 1e-3."""
    a = np.asarray(a, dtype=np.complex128)
    out = np.empty_like(a)
    small = np.abs(a) < 1e-3
    am = a[small]
    out[small] = 1.0 - am / 2.0 + am * am / 6.0 - am * am * am / 24.0
    al = a[~small]
    out[~small] = (1.0 - np.exp(-al)) / al
    return out


def tier(P, i: int, j: int) -> int:
    """|x_i - x_j| < 2 h_j, evaluated as |x_i - x_j|^2 < 4 h_j^2."""
    if i == j:
        return SELF
    if sqnorm(P.centroid[i] - P.centroid[j]) < 4.0 * P.h2[j]:
        return NEAR
    return FAR


def entry_self(P, i: int, s, c: float, n_gl: int = 16):
    """V(s)[i, i].  Duffy-type split of tau_i at x_i into the three sub-triangles
    (x_i, p, q) over its edges.  In polar coordinates about x_i the radial
    integral of U times the area element r dr dtheta is exact:
        int_0^R exp(-s r / c) / (4 pi r) r dr = R phi(s R / c) / (4 pi).
    On the sub-triangle over edge (p, q), with d the distance from x_i to the
    edge line and theta the angle from the perpendicular, R(theta) = d / cos
    theta, and the angular integral over [theta_p, theta_q] is taken with
    n_gl-point Gauss-Legendre."""
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    x = P.centroid[i]
    verts = [P.v0[i], P.v1[i], P.v2[i]]
    v, w = quadrature.gauss_legendre01(n_gl)
    total = np.zeros(s.shape, dtype=np.complex128)
    for e in range(3):
        p, q = verts[e], verts[(e + 1) % 3]
        t = (q - p) / np.linalg.norm(q - p)           # unit edge direction
        tp, tq = np.dot(p - x, t), np.dot(q - x, t)   # tangential coordinates of p, q
        d = np.linalg.norm((p - x) - tp * t)          # distance from x to the edge line
        ta, tb = np.arctan2(tp, d), np.arctan2(tq, d)
        theta = ta + (tb - ta) * v
        R = d / np.cos(theta)                         # (n_gl,)
        vals = R[None, :] * phi(s[:, None] * R[None, :] / c)   # (F, n_gl)
        total += (tb - ta) / FOUR_PI * (vals @ w)
    return total


def entry_quad(x, pts, wts, s, c):
    """sum_q w_q U(|x - y_q|, s) for one collocation point; s may be an array."""
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    r = np.linalg.norm(pts - x[None, :], axis=1)
    return kernel(r[None, :], s[:, None], c) @ wts


def entry(P, i: int, j: int, s, c: float):
    """V(s)[i, j] for every frequency in ``s`` (1D array)."""
    t = tier(P, i, j)
    if t == SELF:
        return entry_self(P, i, s, c)
    if t == NEAR:
        pts, wts = P.near_rule(j)
        return entry_quad(P.centroid[i], pts, wts, s, c)
    return entry_quad(P.centroid[i], P.qp[j], P.qw[j], s, c)


def block(P, rows, cols, s, c: float):
    """Dense entries, shape (len(s), len(rows), len(cols))."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    out = np.zeros((len(s), len(rows), len(cols)), dtype=np.complex128)
    if len(rows) == 0 or len(cols) == 0:
        return out
    x = P.centroid[rows]                                            # (m, 3)
    # far rule everywhere first (vectorised), then overwrite near and self
    # (the far rule's centroid point gives r = 0 on the diagonal; overwritten)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(0, len(rows), 64):
            xa = x[a:a + 64]
            d = xa[:, None, None, :] - P.qp[cols][None, :, :, :]    # (ma, n, 7, 3)
            r = np.sqrt((d * d).sum(-1))                            # (ma, n, 7)
            for f, sf in enumerate(s):
                out[f, a:a + 64, :] = (kernel(r, sf, c) * P.qw[cols][None, :, :]).sum(-1)
    cd2 = sqnorm(x[:, None, :] - P.centroid[cols][None, :, :])
    close = (cd2 < 4.0 * P.h2[cols][None, :]) | (rows[:, None] == cols[None, :])
    for a, b in zip(*np.nonzero(close)):
        out[:, a, b] = entry(P, int(rows[a]), int(cols[b]), s, c)
    return out


def dense(P, s, c: float):
    idx = np.arange(P.n)
    return block(P, idx, idx, s, c)


def galerkin_far(P, rows, cols, s, c: float):
    """Far-field Galerkin entries, shape (len(s), len(rows), len(cols)):
        A^G(s)[i, j] = int_{tau_i} int_{tau_j} U(|x - y|, s) dy dx
    with the 7-point rule on both panels, sum_p sum_q w_ip w_jq U(|y_ip - y_jq|).
    Not the collocation path's operator: the Galerkin variant of the same far
    tier (Sec. 3 names both discretisations; Sec. 2's Galerkin form is
    symmetric), kept for the pin that the far tier's points and weights enter
    both panels alike, A^G = (A^G)^T exactly, and that collocation at the
    centroid is the one-point outer rule of it, |tau_i| V[i, j] ~ A^G[i, j].
    Only meaningful for far pairs (no singular treatment)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    out = np.zeros((len(s), len(rows), len(cols)), dtype=np.complex128)
    for a, i in enumerate(rows):
        # |y_ip - y_jq| for all p (7), all j, all q (7)
        d = P.qp[i][:, None, None, :] - P.qp[cols][None, :, :, :]  # (7, n, 7, 3)
        r = np.sqrt((d * d).sum(-1))
        w = P.qw[i][:, None, None] * P.qw[cols][None, :, :]        # (7, n, 7)
        for f, sf in enumerate(s):
            out[f, a, :] = (kernel(r, sf, c) * w).sum(axis=(0, 2))
    return out
