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
