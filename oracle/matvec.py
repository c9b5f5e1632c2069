"""Products with the frequency-dependent operator (oracle).

Three forms, all over a block partition whose blocks cover every (i, j) once:

  dense            Y[k] = V(s_k) X[k]
  per-frequency H  Y[k] = sum_b A_b(s_k) X[k][J_b], far blocks as U V^H from
                   ACA at the representative frequency, near blocks dense
  compressed       the 3D-ACA form of eq. product: per block
                   A_b(s_k) ~ sum_l f_{b,l}[k] H_{b,l}, so that
                   Y[k]  = sum_b sum_l f_{b,l}[k] H_{b,l} X[k][J_b]   (one column per frequency)
                   y     = sum_k V(s_k) W[k]
                         = sum_b sum_l H_{b,l} ( sum_k f_{b,l}[k] W[k][J_b] )   (eq. product)

For k whose representative is its conjugate partner (freqmap), the
representative operator is applied as conj(V(s_rep) conj(x)).
X, Y, W are (L, n) arrays: one length-n vector per frequency, original order.
"""
from __future__ import annotations

import numpy as np


def dense(A, X):
    """A: (L, n, n) dense operators; X: (L, n)."""
    return np.einsum("kij,kj->ki", A, X)


def _apply_block(data, admissible, x):
    if admissible:
        U, V = data
        return U @ (V.conj().T @ x)
    return data @ x


def hmatrix(blocks, X, rep, conj):
    """blocks: list of (rows, cols, admissible, data) where data[k] holds the
    block at representative frequency k (dense array or (U, V))."""
    L, n = X.shape
    Y = np.zeros((L, n), dtype=np.complex128)
    for k in range(L):
        kr = rep[k]
        x = np.conj(X[k]) if conj[k] else X[k]
        y = np.zeros(n, dtype=np.complex128)
        for rows, cols, adm, data in blocks:
            y[rows] += _apply_block(data[kr], adm, x[cols])
        Y[k] = np.conj(y) if conj[k] else y
    return Y


def compressed(blocks3d, X, rep, conj, kpos):
    """Per-frequency product with the 3D-ACA form.  kpos[k] is the position of
    representative frequency k in the set K the fibers run over."""
    L, n = X.shape
    Y = np.zeros((L, n), dtype=np.complex128)
    for k in range(L):
        p = kpos[rep[k]]
        x = np.conj(X[k]) if conj[k] else X[k]
        y = np.zeros(n, dtype=np.complex128)
        for B in blocks3d:
            xj = x[B.cols]
            acc = np.zeros(len(B.rows), dtype=np.complex128)
            for d in range(B.rank):
                acc += B.fibers[d][p] * _apply_block(B.slices[d], B.admissible, xj)
            y[B.rows] += acc
        Y[k] = np.conj(y) if conj[k] else y
    return Y


def weighted_sum(blocks3d, W, rep, conj, kpos):
    """y = sum_k V(s_k) W[k] by the regrouping of eq. product: the frequency sum
    is taken first, per slice, then each slice is applied once (twice when some
    columns use the conjugate representative)."""
    L, n = W.shape
    y = np.zeros(n, dtype=np.complex128)
    plain = [k for k in range(L) if not conj[k]]
    conjd = [k for k in range(L) if conj[k]]
    for B in blocks3d:
        for d in range(B.rank):
            f = B.fibers[d]
            w1 = np.zeros(len(B.cols), dtype=np.complex128)
            for k in plain:
                w1 += f[kpos[rep[k]]] * W[k][B.cols]
            w2 = np.zeros(len(B.cols), dtype=np.complex128)
            for k in conjd:
                w2 += f[kpos[rep[k]]] * np.conj(W[k][B.cols])
            y[B.rows] += _apply_block(B.slices[d], B.admissible, w1)
            if conjd:
                y[B.rows] += np.conj(_apply_block(B.slices[d], B.admissible, w2))
    return y
