"""Adaptive cross approximation with recompression (oracle; Sec. 4, the
H-matrix face: ACA of admissible blocks followed by QR of both factors and an
SVD of the small core).

The paper cites ACA without fixing the variant.  Reading used (partial
pivoting, as in the cited work):

  approximant  S_k = sum_{l<=k} u_l w_l^T, returned as U V^H with V = conj(W)
  start        row i = 0 (local index), no row used yet
  step k       rho = A[i, :] - sum_l u_l[i] w_l            (row residual)
               j = argmax |rho| (lowest j on ties)
               if rho_j == 0: mark i used, i = lowest unused row, retry
                              (stop when no row is left)
               w_k = rho / rho_j
               u_k = A[:, j] - sum_l w_l[j] u_l            (column residual)
               |S_k|^2 = |S_{k-1}|^2 + 2 Re sum_{l<k} (u_l^H u_k)(w_l^H w_k)
                         + |u_k|^2 |w_k|^2
               stop (keeping term k) if |u_k| |w_k| <= eps max(|S_k|, nu)
               next i = argmax over unused rows of |u_k[i]| (lowest on ties)
  cap          at most min(m, n, max_rank) terms; hitting max_rank first is
               reported as capped.

Recompression: U = Q_U R_U, V = Q_V R_V, R_U R_V^H = Uc S Vc^H (SVD); keep the
smallest t with sqrt(sum_{i>t} s_i^2) <= eps max(sqrt(sum_i s_i^2), nu);
Ubar = Q_U Uc_t S_t, Vbar = Q_V Vc_t, so that U V^H ~ Ubar Vbar^H.

nu is an absolute norm floor, 0 for an ordinary block: both tests are then
relative to the block itself.  The 3D-ACA passes the norm of its current
approximation at the slice's frequency when it compresses a residual slice
(see aca3d).
"""
from __future__ import annotations

import numpy as np


def aca(row_fn, col_fn, m: int, n: int, tol: float, max_rank: int, nu: float = 0.0):
    """row_fn(i) -> A[i, :] (n,), col_fn(j) -> A[:, j] (m,).
    Returns (U (m, k), V (n, k), info dict)."""
    nu_floor = nu
    us, ws = [], []
    used = np.zeros(m, dtype=bool)
    norm2 = 0.0
    i = 0
    capped = False
    kmax = min(m, n)
    rows_evaluated = 0
    while len(us) < kmax:
        if len(us) >= max_rank:
            capped = True
            break
        rho = np.array(row_fn(i), dtype=np.complex128)
        rows_evaluated += 1
        for u, w in zip(us, ws):
            rho -= u[i] * w
        used[i] = True
        j = int(np.argmax(np.abs(rho)))
        if np.abs(rho[j]) == 0.0:
            free = np.nonzero(~used)[0]
            if len(free) == 0:
                break
            i = int(free[0])
            continue
        w = rho / rho[j]
        u = np.array(col_fn(j), dtype=np.complex128)
        for ul, wl in zip(us, ws):
            u -= wl[j] * ul
        cross = 0.0
        for ul, wl in zip(us, ws):
            cross += (np.vdot(ul, u) * np.vdot(wl, w)).real
        n_u, n_w = np.linalg.norm(u), np.linalg.norm(w)
        norm2 = norm2 + 2.0 * cross + (n_u * n_w) ** 2
        us.append(u)
        ws.append(w)
        if n_u * n_w <= tol * max(np.sqrt(max(norm2, 0.0)), nu_floor):
            break
        au = np.abs(u)
        au[used] = -1.0
        if np.all(used):
            break
        i = int(np.argmax(au))
    k = len(us)
    U = np.array(us, dtype=np.complex128).T.reshape(m, k)
    V = np.conj(np.array(ws, dtype=np.complex128)).T.reshape(n, k)
    return U, V, dict(rank=k, capped=capped, norm2=norm2, rows=rows_evaluated)


def recompress(U, V, tol: float, nu: float = 0.0):
    """QR + SVD recompression; returns (Ubar, Vbar, sigma_kept, sigma_all)."""
    m, k = U.shape
    n = V.shape[0]
    if k == 0:
        return U.copy(), V.copy(), np.zeros(0), np.zeros(0)
    QU, RU = np.linalg.qr(U, mode="reduced")
    QV, RV = np.linalg.qr(V, mode="reduced")
    Uc, S, Vch = np.linalg.svd(RU @ RV.conj().T)
    tail = np.sqrt(np.concatenate([np.cumsum((S ** 2)[::-1])[::-1], [0.0]]))  # tail[t] = sqrt(sum_{i>=t} s_i^2)
    total = max(tail[0], nu)
    t = int(np.nonzero(tail <= tol * total)[0][0])
    Ub = QU @ (Uc[:, :t] * S[:t][None, :])
    Vb = QV @ Vch.conj().T[:, :t]
    return Ub, Vb, S[:t], S


def aca_block(P, rows, cols, s, c: float, tol: float, max_rank: int, recompress_tol=None):
    """ACA of the block V(s)[rows, cols] for one frequency, with optional
    recompression at ``recompress_tol``."""
    from . import entries
    rows = np.asarray(rows); cols = np.asarray(cols)
    row_fn = lambda i: entries.block(P, rows[i:i + 1], cols, [s], c)[0, 0, :]
    col_fn = lambda j: entries.block(P, rows, cols[j:j + 1], [s], c)[0, :, 0]
    U, V, info = aca(row_fn, col_fn, len(rows), len(cols), tol, max_rank)
    if recompress_tol is not None:
        U, V, _, _ = recompress(U, V, recompress_tol)
    return U, V, info
