"""3D-ACA of one block over the frequency axis (oracle; Sec. 4, Alg. 1 and
eq. norm, applied per block of the block cluster tree).

The tensor C[i, j, k] = V(s_k)[i, j] over the block (I, J) and the distinct
frequencies K is approximated by sum_l H_l[i, j] f_l[k].  Term l:

  H_l  = V(s_{k_l})[I, J] - sum_{d<l} f_d[k_l] H_d   (residual slice)
         near block: dense; far block: ACA of the residual entry function,
         then QR/SVD recompression (kept as Ubar Vbar^H), both with the
         slice tolerance measured against max(|H_l|, nu_l), where
         nu_l = |sum_{d<l} f_d[k_l] H_d|_F is the current approximation of
         the block at k_l
  (i_l, j_l) = argmax |H_l|   (row-major first on ties; for a far block the
         slice is expanded densely from its factors, as the paper does)
  f_l[k] = (V(s_k)[i_l, j_l] - sum_{d<l} H_d[i_l, j_l] f_d[k]) / H_l[i_l, j_l]
  N^2 += 2 Re sum_{d<l} <H_d, H_l>_F <f_d, f_l> + |H_l|_F^2 |f_l|^2
         with <X, Y> = sum X conj(Y)  (eq. norm, evaluated exactly)
  next frequency k_{l+1} = argmax over k not yet used of |f_l[k]|

Readings of points Alg. 1 leaves open:
  * the loop is always entered; the first frequency is k_1 = K[0];
  * stop when |H_l|_F |f_l| <= eps N; the final rank is then l - 1, i.e. the
    term that met the test is dropped, as the algorithm's final line says;
  * a zero pivot (the residual slice vanishes) stops with rank l - 1;
  * the next frequency is chosen among unused ones (the literal argmax could
    pick k_l again, where |f_l| = 1); when the fiber vanishes at every unused
    frequency, the argmax is undefined and the approximation stops with the
    current terms (the residual fiber through the last pivot is zero there);
  * when every frequency is used, or l reaches r_max, stop keeping term l;
  * the slice tolerance eps_ACA of a residual slice is taken relative to the
    block at that frequency, estimated by nu_l, not relative to the residual
    alone: the residual only has to be resolved to the accuracy the face
    itself is held to (a residual made of the earlier slices' own
    approximation errors has no low-rank structure to find below that level).
"""
from __future__ import annotations

import numpy as np

from . import aca as aca_mod
from . import entries


class Block3D:
    """Result of the 3D-ACA of one block: slices (dense or factored) and fibers."""

    def __init__(self, rows, cols, admissible):
        self.rows = np.asarray(rows)
        self.cols = np.asarray(cols)
        self.admissible = admissible
        self.slices = []      # near: dense (m, n); far: (Ubar, Vbar)
        self.fibers = []      # (|K|,) each
        self.freqs = []       # selected positions in K
        self.capped = False

    @property
    def rank(self):
        return len(self.slices)

    def slice_dense(self, d):
        H = self.slices[d]
        if self.admissible:
            U, V = H
            return U @ V.conj().T
        return H

    def tensor(self):
        """Dense approximant (|K|, m, n)."""
        m, n = len(self.rows), len(self.cols)
        out = np.zeros((len(self.fibers[0]) if self.fibers else 0, m, n), dtype=np.complex128)
        for d in range(self.rank):
            out += self.fibers[d][:, None, None] * self.slice_dense(d)[None, :, :]
        return out


def _inner(X, Y):
    return np.sum(X * np.conj(Y))


def aca3d_block(entry_fn, m: int, n: int, nK: int, admissible: bool, tol_aca: float,
                tol: float, r_max: int, aca_max_rank: int = 10 ** 9, rows=None, cols=None):
    """entry_fn(ri, ci, kpos) -> entries (len(kpos), len(ri), len(ci)) of the
    block for local row/column index arrays and positions in K."""
    B = Block3D(rows if rows is not None else np.arange(m),
                cols if cols is not None else np.arange(n), admissible)
    used = np.zeros(nK, dtype=bool)
    k_cur = 0
    norm2 = 0.0
    Hd = []                   # dense slices (for the pivot expansion and inner products)
    allr, allc = np.arange(m), np.arange(n)
    while True:
        ell = len(B.slices)
        fk = [f[k_cur] for f in B.fibers]
        if admissible:
            approx = np.zeros((m, n), dtype=np.complex128)
            for d in range(ell):
                approx += fk[d] * Hd[d]
            nu = float(np.linalg.norm(approx))

            def row_fn(i):
                r = entry_fn(np.array([i]), allc, [k_cur])[0, 0, :]
                for d in range(ell):
                    U, V = B.slices[d]
                    r = r - fk[d] * (U[i, :] @ V.conj().T)
                return r

            def col_fn(j):
                col = entry_fn(allr, np.array([j]), [k_cur])[0, :, 0]
                for d in range(ell):
                    U, V = B.slices[d]
                    col = col - fk[d] * (U @ V[j, :].conj())
                return col

            U, V, info = aca_mod.aca(row_fn, col_fn, m, n, tol_aca, aca_max_rank, nu=nu)
            Ub, Vb, _, _ = aca_mod.recompress(U, V, tol_aca, nu=nu)
            H = Ub @ Vb.conj().T
            slice_store = (Ub, Vb)
        else:
            H = entry_fn(allr, allc, [k_cur])[0]
            for d in range(ell):
                H = H - fk[d] * Hd[d]
            slice_store = H
        flat = int(np.argmax(np.abs(H)))            # row-major first maximum
        ip, jp = divmod(flat, n)
        piv = H[ip, jp]
        if np.abs(piv) == 0.0:
            break
        fib = entry_fn(np.array([ip]), np.array([jp]), list(range(nK)))[:, 0, 0].astype(np.complex128)
        for d in range(ell):
            fib = fib - Hd[d][ip, jp] * B.fibers[d]
        fib = fib / piv
        used[k_cur] = True
        cross = 0.0
        for d in range(ell):
            cross += (_inner(Hd[d], H) * _inner(B.fibers[d], fib)).real
        nh, nf = np.linalg.norm(H), np.linalg.norm(fib)
        norm2 = norm2 + 2.0 * cross + (nh * nf) ** 2
        if nh * nf <= tol * np.sqrt(max(norm2, 0.0)):
            break                                   # drop this term: rank l - 1
        B.slices.append(slice_store)
        B.fibers.append(fib)
        B.freqs.append(k_cur)
        Hd.append(H)
        if used.all():
            break
        if len(B.slices) >= r_max:
            B.capped = True
            break
        af = np.abs(fib)
        af[used] = -1.0
        if af.max() <= 0.0:
            break
        k_cur = int(np.argmax(af))
    B.norm2 = norm2
    return B


def aca3d_mesh_block(P, rows, cols, s_K, c: float, admissible: bool, tol_aca: float,
                     tol: float, r_max: int):
    """3D-ACA of the block V(s)[rows, cols] over the frequencies s_K."""
    rows = np.asarray(rows); cols = np.asarray(cols)
    s_K = np.asarray(s_K)

    def entry_fn(ri, ci, kpos):
        return entries.block(P, rows[ri], cols[ci], s_K[list(kpos)], c)

    return aca3d_block(entry_fn, len(rows), len(cols), len(s_K), admissible, tol_aca, tol,
                       r_max, rows=rows, cols=cols)
