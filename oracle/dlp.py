"""Laplace-domain double-layer entries (oracle).

Test infrastructure: imported only by the tests, the smoke check and the
benchmark's CPU baseline.  Plain float64/complex128 numpy.

K(s)[i, j] = integral over tau_j of the normal derivative (in y, outward unit
normal n_y) of the transformed fundamental solution U(x_i - y, s) (Sec. 2,
eq. dlp, with every kernel replaced by its transform as in Sec. 3).  With
kappa = s / c, d = x - y and r = |d|,

    d/dn_y U = (d . n_y) (1 + kappa r) exp(-kappa r) / (4 pi r^3).

Reading used: the paper pairs the double layer with linear continuous trial
functions; here, as for the single layer, densities are piecewise constant
and collocated at the centroids, so the matrix has the single layer's shape
and tiers:

  self  (i == j)              0: the collocation point lies in the plane of the
                              flat panel, where d . n_y vanishes.
  near  (|x_i - x_j| < 2 h_j) 7-point rule on 16 sub-triangles (112 points).
  far   (otherwise)           7-point rule.
"""
from __future__ import annotations

import math

import numpy as np

from .entries import NEAR, SELF, tier
from .geometry import sqnorm

FOUR_PI = 4.0 * math.pi


def kernel_dn(d, n, s, c):
    """Normal derivative of U for separations d (..., 3) and normals n (..., 3)
    (broadcast), at one complex frequency s."""
    r = np.sqrt((d * d).sum(-1))
    dn = (d * n).sum(-1)
    k = s / c
    return dn * (1.0 + k * r) * np.exp(-k * r) / (FOUR_PI * r ** 3)


def entry(P, i: int, j: int, s, c: float):
    """K(s)[i, j] for every frequency in ``s`` (1D array)."""
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    t = tier(P, i, j)
    if t == SELF:
        return np.zeros(s.shape, dtype=np.complex128)
    if t == NEAR:
        pts, wts = P.near_rule(j)
    else:
        pts, wts = P.qp[j], P.qw[j]
    d = P.centroid[i][None, :] - pts
    return np.array([kernel_dn(d, P.normal[j][None, :], sf, c) @ wts for sf in s])


def block(P, rows, cols, s, c: float):
    """Dense entries, shape (len(s), len(rows), len(cols))."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    out = np.zeros((len(s), len(rows), len(cols)), dtype=np.complex128)
    if len(rows) == 0 or len(cols) == 0:
        return out
    x = P.centroid[rows]
    nrm = P.normal[cols][None, :, None, :]                          # (1, n, 1, 3)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(0, len(rows), 64):
            d = x[a:a + 64][:, None, None, :] - P.qp[cols][None, :, :, :]   # (ma, n, 7, 3)
            for f, sf in enumerate(s):
                out[f, a:a + 64, :] = (kernel_dn(d, nrm, sf, c) * P.qw[cols][None, :, :]).sum(-1)
    cd2 = sqnorm(x[:, None, :] - P.centroid[cols][None, :, :])
    close = (cd2 < 4.0 * P.h2[cols][None, :]) | (rows[:, None] == cols[None, :])
    for a, b in zip(*np.nonzero(close)):
        out[:, a, b] = entry(P, int(rows[a]), int(cols[b]), s, c)
    return out


def dense(P, s, c: float):
    idx = np.arange(P.n)
    return block(P, idx, idx, s, c)


def sphere_constant(R: float, s, c: float):
    """Closed form of the double layer of the constant density 1 on a sphere of
    radius R, at a point of the sphere: with kappa = s / c,
        -(1 - exp(-2 kappa R) (1 + kappa R)) / (2 kappa R)
    (-1/2 as kappa -> 0, Gauss's solid-angle identity).  For x on the sphere the
    points y at distance r carry the area 2 pi r dr and d . n_y = -r^2 / (2R),
    so the integral is -(1 / 4R) int_0^{2R} (1 + kappa r) exp(-kappa r) dr."""
    k = np.asarray(s, dtype=np.complex128) / c
    a = k * R
    # 1 - exp(-2a)(1 + a) = -expm1(-2a) - a exp(-2a), without the cancellation at small a
    return (np.expm1(-2.0 * a) + a * np.exp(-2.0 * a)) / (2.0 * a)
