"""FMM-based 3D-ACA (oracle; Sec. 4, the face approximated by a black-box
FMM, eq. cheb; Alg. 1 and eq. norm along the frequency axis).

Test infrastructure: only the tests, the package's smoke check and the
benchmark's CPU baseline use this module; the library never does.

The far field of an admissible block (X, Y) is not built from ACA factors
but from Chebyshev interpolation of the kernel in both clusters' boxes:

  U(x, y, s) ~ sum_n S_X(x, x_n) sum_m U(x_n, y_m, s) S_Y(y, y_m)      (eq. cheb)

so that the block of collocation entries is

  A_XY(s) ~ L_X K_XY(s) R_Y^T,
    L_X[i, n]  = S_X(x_i, x_n)                      (x_i: collocation point of panel i)
    R_Y[j, m]  = sum_q w_jq S_Y(y_jq, y_m)          (the panels' far rule, weights with area)
    K_XY(s)[n, m] = U(x_n, y_m, s) = exp(-s r / c) / (4 pi r),  r = |x_n - y_m|

Only the M2L operator K_XY(s) depends on the frequency; Alg. 1 compresses the
tensor [K_XY(s_k)]_k over the frequencies of K with dense slices (the
"relevant entries" of the FMM variant are those of the M2L operators).  Near
blocks are compressed exactly as in the H-matrix variant (dense slices of V).

Readings (the paper names the method, not these details):
  * order p = number of Chebyshev nodes per dimension, t_a = cos((2a+1) pi/(2p)),
    a = 0..p-1 (the zeros of T_p), interpolation by polynomials of degree
    p - 1 in each coordinate; nodes of a box numbered n = a_x + p a_y + p^2 a_z;
    S_X is the tensor product of the 1D Lagrange polynomials of these nodes;
  * the box of a cluster is the axis-aligned box of its triangles' vertices
    (the box the admissibility condition eq. admissible is evaluated on), so
    that collocation and quadrature points lie inside it; a half-width below
    1e-3 of the box's largest half-width is raised to that value (a flat
    cluster would otherwise give coinciding nodes);
  * the cluster tree and block tree are the H-matrix variant's (the paper's
    uniform octree only changes which clusters pair up; any cluster tree with
    boxes serves the interpolation);
  * the multi-level evaluation (P2M, M2M, M2L, L2L, L2P) gives the same
    product as this single-level definition: the parent's Lagrange
    polynomials are interpolated exactly by the son's nodes (degree p - 1),
    so R_P = [R_son T_son] and L_P likewise, with
    T_son[m, m'] = S_P(y_m^son, y_m'^P).
"""
from __future__ import annotations

import numpy as np

from . import aca3d as aca3d_mod
from .tree import ClusterTree

FOUR_PI = 4.0 * np.pi
MIN_HALF_WIDTH = 1e-3


def cheb_nodes(p: int):
    """Zeros of T_p on [-1, 1]: t_a = cos((2a + 1) pi / (2p))."""
    a = np.arange(p)
    return np.cos((2 * a + 1) * np.pi / (2 * p))


def lagrange_1d(t, p: int):
    """Values (len(t), p) of the Lagrange polynomials of the p Chebyshev nodes."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    nodes = cheb_nodes(p)
    out = np.ones((len(t), p))
    for a in range(p):
        for b in range(p):
            if b != a:
                out[:, a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return out


def box_of(T: ClusterTree, c: int):
    """(centre, half-widths) of cluster c's interpolation box."""
    lo, hi = np.asarray(T.bmin[c], np.float64), np.asarray(T.bmax[c], np.float64)
    centre = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    half = np.maximum(half, MIN_HALF_WIDTH * half.max())
    return centre, half


def box_nodes(box, p: int):
    """The p^3 Chebyshev nodes of a box, (p^3, 3), n = a_x + p a_y + p^2 a_z."""
    centre, half = box
    t = cheb_nodes(p)
    az, ay, ax = np.meshgrid(np.arange(p), np.arange(p), np.arange(p), indexing="ij")
    idx = np.stack([ax.ravel(), ay.ravel(), az.ravel()], axis=1)
    return centre[None, :] + half[None, :] * t[idx]


def interp(box, pts, p: int):
    """S(pts, x_n) for all nodes n of the box: (len(pts), p^3)."""
    centre, half = box
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    u = (pts - centre[None, :]) / half[None, :]
    lx, ly, lz = (lagrange_1d(u[:, d], p) for d in range(3))
    return (lz[:, :, None, None] * ly[:, None, :, None] * lx[:, None, None, :]).reshape(len(pts), p ** 3)


def l_op(P, box, rows, p: int):
    """L_X: interpolation at the collocation points (centroids) of rows."""
    return interp(box, P.centroid[np.asarray(rows)], p)


def r_op(P, box, cols, p: int):
    """R_Y: the far rule of each panel applied to the box's Lagrange polynomials."""
    cols = np.asarray(cols)
    q = P.qp[cols].reshape(-1, 3)
    S = interp(box, q, p).reshape(len(cols), P.qp.shape[1], p ** 3)
    return np.einsum("jq,jqm->jm", P.qw[cols], S)


def transfer(son_box, parent_box, p: int):
    """T_son[m, m'] = S_P(y_m^son, y_m'^P): (p^3, p^3)."""
    return interp(parent_box, box_nodes(son_box, p), p)


def m2l(boxX, boxY, s, c: float, p: int):
    """K_XY(s) for each frequency of s: (len(s), p^3, p^3)."""
    s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
    xn, ym = box_nodes(boxX, p), box_nodes(boxY, p)
    d = xn[:, None, :] - ym[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    return np.exp(-s[:, None, None] * r[None, :, :] / c) / (FOUR_PI * r[None, :, :])


def far_block_dense(P, T, X: int, Y: int, s, c: float, p: int):
    """The interpolated block L_X K_XY(s) R_Y^T at each frequency: (len(s), |X|, |Y|)."""
    bx, by = box_of(T, X), box_of(T, Y)
    L = l_op(P, bx, T.indices(X), p)
    R = r_op(P, by, T.indices(Y), p)
    K = m2l(bx, by, s, c, p)
    return np.einsum("in,knm,jm->kij", L, K, R)


class FmmBlock:
    """3D-ACA of an admissible block's M2L tensor: dense p^3 x p^3 slices."""

    def __init__(self, rows, cols, L, R, b3):
        self.rows, self.cols = np.asarray(rows), np.asarray(cols)
        self.L, self.R, self.b3 = L, R, b3

    @property
    def rank(self):
        return self.b3.rank


def fmm3d_far_block(P, T, X: int, Y: int, s_K, c: float, p: int, tol: float, r_max: int):
    """Alg. 1 on the tensor [K_XY(s_k)]_k with dense residual slices."""
    bx, by = box_of(T, X), box_of(T, Y)
    s_K = np.asarray(s_K)
    K = m2l(bx, by, s_K, c, p)

    def entry_fn(ri, ci, kpos):
        return K[np.asarray(list(kpos))][:, ri][:, :, ci]

    b3 = aca3d_mod.aca3d_block(entry_fn, p ** 3, p ** 3, len(s_K), False, 0.0, tol, r_max)
    return FmmBlock(T.indices(X), T.indices(Y), l_op(P, bx, T.indices(X), p),
                    r_op(P, by, T.indices(Y), p), b3)


def fmm3d(P, T, B, s_K, c: float, p: int, tol: float, r_max: int):
    """Per block of the partition B: far blocks as FmmBlock, near blocks as the
    H-matrix variant's dense 3D-ACA (Block3D)."""
    out = []
    for X, Y, adm in B:
        if adm:
            out.append(fmm3d_far_block(P, T, X, Y, s_K, c, p, tol, r_max))
        else:
            out.append(aca3d_mod.aca3d_mesh_block(P, T.indices(X), T.indices(Y), s_K, c, False,
                                                  0.0, tol, r_max))
    return out


def product(blocks, X, rep, conj, kpos):
    """Per-frequency product with the FMM-based 3D-ACA (the single-level form):
    far blocks apply L_X (sum_d f_d[k] H_d) R_Y^T, near blocks sum_d f_d[k] H_d.
    Conjugate-represented columns as in matvec.compressed."""
    L, n = X.shape
    Y = np.zeros((L, n), dtype=np.complex128)
    for k in range(L):
        kp = kpos[rep[k]]
        x = np.conj(X[k]) if conj[k] else X[k]
        y = np.zeros(n, dtype=np.complex128)
        for Bk in blocks:
            if isinstance(Bk, FmmBlock):
                w = Bk.R.T @ x[Bk.cols]
                z = np.zeros(Bk.L.shape[1], dtype=np.complex128)
                for d in range(Bk.b3.rank):
                    z += Bk.b3.fibers[d][kp] * (Bk.b3.slices[d] @ w)
                y[Bk.rows] += Bk.L @ z
            else:
                xj = x[Bk.cols]
                for d in range(Bk.rank):
                    y[Bk.rows] += Bk.fibers[d][kp] * (Bk.slices[d] @ xj)
        Y[k] = np.conj(y) if conj[k] else y
    return Y
