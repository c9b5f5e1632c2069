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


@pytest.mark.parametrize("m", [1, 2, 3])
def test_radau_iia_tableaux(m):
    """Order conditions of Radau IIA (c = A 1, b^T A^{-1} = (0,..,0,1), c_m = 1)
    and the stage order: A c^{k-1} = c^k / k for k <= m."""
    A = gcq.radau_iia(m)
    c = A @ np.ones(m)
    b = A[-1]
    assert abs(c[-1] - 1.0) < 1e-14
    e = np.zeros(m)
    e[-1] = 1.0
    assert np.max(np.abs(b @ np.linalg.inv(A) - e)) < 1e-13
    for k in range(1, m + 1):
        assert np.max(np.abs(A @ c ** (k - 1) - c ** k / k)) < 1e-13


@pytest.mark.parametrize("m", [2, 3])
def test_rk_scheme_reproduces_radau_iia(m):
    """V = 1/(s + lam): the gCQ stage values are those of Radau IIA applied to
    f' = -lam f + q: F_n = (I + lam dt A)^{-1} (f_{n-1} 1 + dt A Q_n), f_n the
    last stage; V = s: stage derivatives (dt A)^{-1} (Q_n - q_{n-1} 1)."""
    A = gcq.radau_iia(m)
    rng = np.random.default_rng(13)
    N = 14
    dt = 0.01 * (1.0 + 3.0 * rng.random(N))
    s, w = contour.contour(101 if m == 2 else 301, *gcq.contour_steps(A, dt.min(), dt.max()))
    q = rng.standard_normal((N, m, 3))
    lam = 40.0
    f = gcq.convolve_rk(lambda z, X: X / (z + lam), A, q, dt, s, w)
    prev = np.zeros(3)
    ref = np.zeros_like(q)
    for n in range(N):
        F = np.linalg.solve(np.eye(m) + lam * dt[n] * A, np.outer(np.ones(m), prev) + dt[n] * (A @ q[n]))
        ref[n] = F
        prev = F[-1]
    assert np.max(np.abs(f - ref)) <= 1e-9 * np.max(np.abs(ref))
    d = gcq.convolve_rk(lambda z, X: z * X, A, q, dt, s, w)
    qprev = np.zeros(3)
    for n in range(N):
        dref = np.linalg.solve(dt[n] * A, q[n] - np.outer(np.ones(m), qprev))
        assert np.max(np.abs(d[n] - dref)) <= 1e-8 * np.max(np.abs(dref)), n
        qprev = q[n, -1]


@pytest.mark.parametrize("m", [2, 3])
def test_rk_long_run_with_the_papers_point_count(m):
    """60 variable steps with N_Q = N (ln N)^2 points (App. A): the stage values
    of Radau IIA for V = 1/(s + lam).  On this contour |R(dt s)| exceeds 1 at some
    points (2.9 for two stages), so the quadrature must resolve the cancellation:
    with a fixed, small N_Q long runs diverge, with the paper's count they do not."""
    A = gcq.radau_iia(m)
    rng = np.random.default_rng(17)
    N = 60
    dt = 0.01 * (1.0 + 3.0 * rng.random(N))
    s, w = contour.contour(contour.n_points(N, m) + 1, *gcq.contour_steps(A, dt.min(), dt.max()))
    q = rng.standard_normal((N, m, 2))
    lam = 40.0
    f = gcq.convolve_rk(lambda z, X: X / (z + lam), A, q, dt, s, w)
    prev = np.zeros(2)
    ref = np.zeros_like(q)
    for n in range(N):
        ref[n] = np.linalg.solve(np.eye(m) + lam * dt[n] * A, np.outer(np.ones(m), prev) + dt[n] * (A @ q[n]))
        prev = ref[n, -1]
    assert np.max(np.abs(f - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_rk_one_stage_is_implicit_euler_scheme():
    dt, s, w, q = _setup(12, seed=14)
    V = lambda z, X: X / (z + 25.0)
    f1 = gcq.convolve(V, q, dt, s, w)
    fr = gcq.convolve_rk(V, gcq.radau_iia(1), q[:, None, :], dt, s, w)[:, 0, :]
    assert np.max(np.abs(f1 - fr)) <= 1e-12 * np.max(np.abs(f1))


def test_stability_interval_ends():
    """x* of R(x) = e_m^T (I - x A)^{-1} 1: implicit Euler 1/(1 - x) has |R| > 1
    on (0, 2); 2-stage Radau IIA (1 + x/3) / (1 - 2x/3 + x^2/6) on (0, 6)."""
    assert abs(gcq.stability_end(gcq.radau_iia(1)) - 2.0) < 1e-9
    assert abs(gcq.stability_end(gcq.radau_iia(2)) - 6.0) < 1e-9
    x3 = gcq.stability_end(gcq.radau_iia(3))
    R = lambda x: np.linalg.solve(np.eye(3) - x * gcq.radau_iia(3), np.ones(3))[-1]
    assert abs(abs(R(x3)) - 1.0) < 1e-9 and abs(R(x3 * 1.01)) < 1.0 < abs(R(x3 * 0.99))


@pytest.mark.parametrize("m", [2, 3])
def test_rk_contour_keeps_the_growth_small(m):
    """On the contour of the reading, |R(dt_min s_l)| stays below 1.5 (the
    printed scaling reaches 2.9 for two stages and 9 for three)."""
    A = gcq.radau_iia(m)
    s, _ = contour.contour(401, *gcq.contour_steps(A, 0.01, 0.03))
    R = [abs(np.linalg.solve(np.eye(m) - 0.01 * z * A, np.ones(m))[-1]) for z in s]
    assert max(R) < 1.5
