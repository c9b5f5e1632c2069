"""Generalised convolution quadrature of a convolution f = V * q (oracle;
Sec. 3, temporal discretisation: the first step, eq. gCQ_xn and
eq. gcq_formula), with implicit Euler as the underlying Runge-Kutta method.

Test infrastructure: imported only by the tests, the smoke check and the
benchmark's CPU baseline.  Plain float64/complex128 numpy.

Implicit Euler is the one-stage method A = (1), b = c = (1), for which
b^T A^{-1} = 1 and the stage vectors are the nodal vectors.  With steps
dt_1..dt_N, contour points s_l and weights w_l (App. A) and V(z) the Laplace-
domain operator:

  f_1 = V(1/dt_1) q_1                                         (zero initial state)
  for n = 2..N:
    x_{n-1}(s_l) = (x_{n-2}(s_l) + dt_{n-1} q_{n-1}) / (1 - dt_{n-1} s_l),  x_0 = 0
    f_n = V(1/dt_n) q_n + sum_l V(s_l) w_l x_{n-1}(s_l) / (1 - dt_n s_l)

The weights are those of oracle.contour (the contour traversed clockwise,
sum_l w_l g(s_l) ~ -(1/2 pi i) times the counter-clockwise integral); with
them the scheme reproduces implicit Euler for V(s) = 1/(s + lam), s and s^2,
which the tests check.  The contour passes through s = 0 (gamma(-K + i K'/2)
= 0) and 2/dt_min; V must be analytic on and inside it (the wave kernel
exp(-s r)/(4 pi r) is entire in s).
"""
from __future__ import annotations

import numpy as np


def convolve(apply_V, q, dt, s, w):
    """f (N, M) complex from q (N, M), dt (N,), contour s, w (N_Q,).
    apply_V(z, X) returns V(z) X for a complex scalar z and a vector X (M,)."""
    q = np.asarray(q, dtype=np.complex128)
    dt = np.asarray(dt, dtype=np.float64)
    s = np.asarray(s, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    N, M = q.shape
    x = np.zeros((len(s), M), dtype=np.complex128)
    f = np.zeros((N, M), dtype=np.complex128)
    f[0] = apply_V(1.0 / dt[0], q[0])
    for n in range(1, N):            # paper step n + 1
        x = (x + dt[n - 1] * q[n - 1][None, :]) / (1.0 - dt[n - 1] * s)[:, None]
        acc = apply_V(1.0 / dt[n], q[n])
        for l in range(len(s)):
            acc = acc + apply_V(s[l], w[l] * x[l] / (1.0 - dt[n] * s[l]))
        f[n] = acc
    return f


def solve(apply_V, solve_V, f, dt, s, w):
    """q (N, M) with convolve(apply_V, q, dt, s, w) = f (eq. gcq_formula with
    (f)_n given): per step the system V(1/dt_n) q_n = f_n - history, the
    history being the contour sum of eq. gcq_formula over the earlier steps.
    solve_V(z, b) returns V(z)^{-1} b."""
    f = np.asarray(f, dtype=np.complex128)
    dt = np.asarray(dt, dtype=np.float64)
    s = np.asarray(s, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    N, M = f.shape
    x = np.zeros((len(s), M), dtype=np.complex128)
    q = np.zeros((N, M), dtype=np.complex128)
    for n in range(N):
        h = np.zeros(M, dtype=np.complex128)
        if n > 0:
            x = (x + dt[n - 1] * q[n - 1][None, :]) / (1.0 - dt[n - 1] * s)[:, None]
            for l in range(len(s)):
                h = h + apply_V(s[l], w[l] * x[l] / (1.0 - dt[n] * s[l]))
        q[n] = solve_V(1.0 / dt[n], f[n] - h)
    return q


# ---- Runge-Kutta methods of m stages ------------------------------------------
# The paper's scheme for an A- and L-stable method (c | A, b^T) with
# b^T A^{-1} = (0, .., 0, 1): quantities per node carry the m stage values;
# V((dt A)^{-1}) acts through the eigendecomposition (dt A)^{-1} = P diag(lam) P^{-1}
# as P diag(V(lam_e)) P^{-1}; b^T A^{-1} x picks the last stage.

def radau_iia(m: int):
    """Butcher matrix A of the Radau IIA method with m = 1, 2 or 3 stages."""
    if m == 1:
        return np.array([[1.0]])
    if m == 2:
        return np.array([[5.0 / 12.0, -1.0 / 12.0], [0.75, 0.25]])
    if m == 3:
        r = np.sqrt(6.0)
        return np.array([[(88 - 7 * r) / 360, (296 - 169 * r) / 1800, (-2 + 3 * r) / 225],
                         [(296 + 169 * r) / 1800, (88 + 7 * r) / 360, (-2 - 3 * r) / 225],
                         [(16 - r) / 36, (16 + r) / 36, 1.0 / 9.0]])
    raise ValueError("m must be 1, 2 or 3")


def stability_end(A) -> float:
    """Right end x* of the interval (0, x*) of the positive real axis on which
    the method's stability function R(x) = e_m^T (I - x A)^{-1} 1 exceeds 1 in
    modulus (x* = 2 for implicit Euler, 6 for 2-stage Radau IIA): a grid search
    for the last sign change of |R| - 1, refined by bisection."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    one = np.ones(m)
    g = lambda x: abs(np.linalg.solve(np.eye(m) - x * A, one)[-1]) - 1.0
    xs = np.linspace(1e-6, 200.0, 20001)
    vals = np.array([g(x) for x in xs])
    i = int(np.nonzero(vals > 0)[0].max())
    lo, hi = xs[i], xs[i + 1]
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if g(mid) > 0 else (lo, mid)
    return 0.5 * (lo + hi)


def contour_steps(A, dt_min: float, dt_max: float):
    """Arguments (dt_min, dt_max, stage_ratio) of oracle.contour for method A.

    Reading of App. A for m > 1 stages.  The printed q = 5 dt_max max|lambda(A)| /
    (dt_min min|lambda(A)|) is kept (stage_ratio = 5 max|lambda| / min|lambda|).
    The contour always crosses the real axis at 0 and 2 / (dt_min scale); the
    printed scale (the step itself) puts the crossing inside the interval
    (0, x*/dt_min) where the stability function grows (|R(dt s)| > 1), and the
    states at those points grow step by step until rounding swamps the
    quadrature (Radau IIA with 3 stages diverges within 100 steps).  The
    reading scales gamma by dt_min / x* instead, so the crossing is at
    2 x* / dt_min, twice the end of that interval; with N_Q = N (log N)^2 points
    it reproduces Radau IIA over long runs (tests).  One stage (implicit Euler):
    the printed contour, (dt_min, dt_max, 1)."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape[0] == 1:
        return dt_min * A[0, 0], dt_max * A[0, 0], 1.0
    ev = np.abs(np.linalg.eigvals(A))
    x = stability_end(A)
    return dt_min / x, dt_max / x, 5.0 * ev.max() / ev.min()


def _matrix_V(apply_V, Z, Qs):
    lam, P = np.linalg.eig(Z)
    R = np.linalg.solve(P, Qs)
    return P @ np.stack([apply_V(lam[e], R[e]) for e in range(len(lam))])


def convolve_rk(apply_V, A, q, dt, s, w):
    """Stage values f (N, m, M) from stage values q (N, m, M): the first step
    f_1 = V((dt_1 A)^{-1}) q_1, then eq. gCQ_xn and eq. gcq_formula."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    q = np.asarray(q, dtype=np.complex128)
    dt = np.asarray(dt, dtype=np.float64)
    N, _, M = q.shape
    one = np.ones(m)
    I = np.eye(m)
    x = np.zeros((len(s), m, M), dtype=np.complex128)
    f = np.zeros((N, m, M), dtype=np.complex128)
    f[0] = _matrix_V(apply_V, np.linalg.inv(dt[0] * A), q[0])
    for n in range(1, N):
        for l in range(len(s)):
            rhs = np.outer(one, x[l, m - 1]) + dt[n - 1] * (A @ q[n - 1])
            x[l] = np.linalg.solve(I - dt[n - 1] * s[l] * A, rhs)
        acc = _matrix_V(apply_V, np.linalg.inv(dt[n] * A), q[n])
        for l in range(len(s)):
            u = np.linalg.solve(I - dt[n] * s[l] * A, one)
            W = w[l] * np.outer(u, x[l, m - 1])
            acc = acc + np.stack([apply_V(s[l], W[i]) for i in range(m)])
        f[n] = acc
    return f
