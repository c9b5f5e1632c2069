"""Restarted GMRES (oracle).

The paper solves each time step's system with unpreconditioned BiCGstab to the
ACA precision (Sec. 5).  The library's solver step is restarted GMRES(m) run on
every frequency's system at once; the oracle is the textbook algorithm, one
system at a time:

  x0 = 0; repeat cycles:
    r = b - A x (true residual); stop if |r| <= rtol |b|
    v_1 = r / |r|; for j = 1..m:
      w = A v_j; classical Gram-Schmidt applied twice against v_1..v_j;
      h_{j+1,j} = |w|; v_{j+1} = w / h_{j+1,j}
      Givens rotations reduce H to upper triangular; |g_{j+1}| is the
      residual norm of the least-squares problem; stop the cycle early if
      it falls to rtol |b|
    x += V_m y with R y = g
"""
from __future__ import annotations

import numpy as np


def gmres(apply_A, b, rtol: float = 1e-6, restart: int = 50, max_iter: int = 1000):
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, dict(iters=0, resid=0.0, converged=True)
    iters = 0
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * nb or iters >= max_iter:
            return x, dict(iters=iters, resid=beta / nb, converged=beta <= rtol * nb)
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.float64)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        jdone = 0
        for j in range(m):
            w = apply_A(V[j])
            h = V[:j + 1].conj() @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1].conj() @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            H[:j + 1, j] = h
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            if hn > 0:
                V[j + 1] = w / hn
            for i in range(j):           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                if abs(a) == 0:
                    cs[j], sn[j] = 0.0, 1.0 * np.conj(bb) / abs(bb)
                else:
                    cs[j] = abs(a) / den
                    sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            jdone = j + 1
            if abs(g[j + 1]) <= rtol * nb or hn == 0 or iters >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:jdone, :jdone]), g[:jdone])
        x = x + V[:jdone].T @ y
