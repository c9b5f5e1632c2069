"""Pins of the gCQ stepping oracle (Sec. 3, eq. gCQ_xn, eq. gcq_formula; App. A
contour): with implicit Euler as the underlying method the scheme must
reproduce implicit Euler applied to the ODE behind each scalar operator --
an exponential kernel (V = 1/(s + lam)), differentiation (V = s) and the
second derivative (V = s^2) -- on variable steps, converging spectrally in
the number of contour points.  (The contour passes through s = 0, so an
operator with a pole there, such as 1/s, is outside the method's reach.)"""
import numpy as np
import pytest

from oracle import contour, gcq


def _setup(N, n_q=81, seed=0):
    rng = np.random.default_rng(seed)
    dt = 0.01 * (1.0 + 3.0 * rng.random(N))          # dt in [0.01, 0.04]
    s, w = contour.contour(n_q, dt.min(), dt.max() * 1.0001)
    q = np.random.default_rng(seed + 1).standard_normal((N, 3))
    return dt, s, w, q


def _euler_exponential(q, dt, lam):
    ref = np.zeros_like(q)
    prev = np.zeros(q.shape[1])
    for n in range(len(dt)):                           # f' = -lam f + q
        prev = (prev + dt[n] * q[n]) / (1.0 + lam * dt[n])
        ref[n] = prev
    return ref


@pytest.mark.parametrize("lam", [20.0, 100.0])
def test_exponential_kernel_gives_implicit_euler(lam):
    dt, s, w, q = _setup(25, seed=2)
    f = gcq.convolve(lambda z, X: X / (z + lam), q, dt, s, w)
    ref = _euler_exponential(q, dt, lam)
    assert np.max(np.abs(f - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_spectral_convergence_in_the_number_of_points():
    lam = 5.0
    errs = []
    for n_q in (41, 81, 161):
        dt, s, w, q = _setup(25, n_q=n_q, seed=2)
        f = gcq.convolve(lambda z, X: X / (z + lam), q, dt, s, w)
        ref = _euler_exponential(q, dt, lam)
        errs.append(np.max(np.abs(f - ref)) / np.max(np.abs(ref)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-10


def test_differentiation_operators_give_backward_differences():
    dt, s, w, q = _setup(20, seed=4)
    f1 = gcq.convolve(lambda z, X: z * X, q, dt, s, w)
    qp = np.vstack([np.zeros(q.shape[1]), q[:-1]])
    d1 = (q - qp) / dt[:, None]                        # zero initial value
    assert np.max(np.abs(f1 - d1)) <= 1e-10 * np.max(np.abs(d1))
    f2 = gcq.convolve(lambda z, X: z * z * X, q, dt, s, w)
    d1p = np.vstack([np.zeros(q.shape[1]), d1[:-1]])
    d2 = (d1 - d1p) / dt[:, None]
    assert np.max(np.abs(f2 - d2)) <= 1e-9 * np.max(np.abs(d2))


def test_linearity_and_zero_input():
    dt, s, w, q = _setup(10, seed=6)
    V = lambda z, X: X / (z + 50.0)
    f1 = gcq.convolve(V, q, dt, s, w)
    f2 = gcq.convolve(V, 2.0 * q, dt, s, w)
    assert np.max(np.abs(f2 - 2.0 * f1)) <= 1e-12 * np.max(np.abs(f1))
    assert np.all(gcq.convolve(V, np.zeros_like(q), dt, s, w) == 0)


def test_solve_inverts_implicit_euler_of_the_exponential_kernel():
    """V = 1/(s + lam): f_n = (f_{n-1} + dt_n q_n) / (1 + lam dt_n), so
    q_n = ((1 + lam dt_n) f_n - f_{n-1}) / dt_n."""
    lam = 40.0
    dt, s, w, f = _setup(20, seed=8)
    q = gcq.solve(lambda z, X: X / (z + lam), lambda z, b: b * (z + lam), f, dt, s, w)
    fp = np.vstack([np.zeros(f.shape[1]), f[:-1]])
    ref = ((1.0 + lam * dt[:, None]) * f - fp) / dt[:, None]
    assert np.max(np.abs(q - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_solve_and_convolve_are_inverse_for_a_matrix_operator():
    rng = np.random.default_rng(9)
    M = 6
    A0 = rng.standard_normal((M, M)) / M
    V = lambda z, X: np.linalg.solve(z * np.eye(M) + 30.0 * np.eye(M) + A0, X)   # resolvent-like, analytic
    Vinv = lambda z, b: (z * np.eye(M) + 30.0 * np.eye(M) + A0) @ b
    dt, s, w, _ = _setup(15, seed=10)
    q = rng.standard_normal((15, M))
    f = gcq.convolve(V, q, dt, s, w)
    q2 = gcq.solve(V, Vinv, f, dt, s, w)
    assert np.max(np.abs(q2 - q)) <= 1e-9 * np.max(np.abs(q))
