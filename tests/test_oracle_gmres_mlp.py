"""Pins of the oracle's GMRES (against LAPACK's direct solve) and of the MLP
(central finite differences of the loss, a decreasing training loss, and the
Adam update against its closed form after one step)."""
import numpy as np

from oracle import entries, gmres, mlp
from oracle.geometry import Panels
from synth import freq, mesh, rhs


def test_gmres_matches_direct_solve():
    xyz, tri = mesh.icosphere(2)
    P = Panels(xyz, tri)
    s = freq.bdf2_circle(32, 0.05, 1e-8 ** (1 / 32))[[0, 5, 16]]
    A = entries.dense(P, s, 1.0)
    B = rhs.random_complex(len(s), P.n, 1)
    for k in range(len(s)):
        x, info = gmres.gmres(lambda v: A[k] @ v, B[k], rtol=1e-10, restart=20, max_iter=500)
        xs = np.linalg.solve(A[k], B[k])
        assert info["converged"]
        assert np.linalg.norm(A[k] @ x - B[k]) <= 1e-10 * np.linalg.norm(B[k]) * 1.01
        assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_gmres_restart_and_zero_rhs():
    rng = np.random.default_rng(0)
    n = 60
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n) + 0j
    b = rng.standard_normal(n) + 0j
    x, info = gmres.gmres(lambda v: A @ v, b, rtol=1e-12, restart=5, max_iter=400)
    assert info["converged"] and info["iters"] > 5
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9)
    x, info = gmres.gmres(lambda v: A @ v, np.zeros(n, complex))
    assert info["iters"] == 0 and not x.any()


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(0)
    theta = mlp.glorot_init(0) + 0.05 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((32, 5))
    t = rng.standard_normal(32)
    _, g = mlp.loss_and_grad(theta, X, t)
    h = 1e-6
    for idx in rng.choice(mlp.N_PARAMS, 40, replace=False):
        e = np.zeros(mlp.N_PARAMS); e[idx] = h
        lp, _ = mlp.loss_and_grad(theta + e, X, t)
        lm, _ = mlp.loss_and_grad(theta - e, X, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(g[idx]))


def test_mlp_training_decreases_loss_and_adam_first_step():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((256, 5))
    t = np.tanh(X[:, 0]) + 0.5 * X[:, 1]
    theta = mlp.glorot_init(0)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    l0, g = mlp.loss_and_grad(theta, X, t)
    # after bias correction the first Adam step is lr * g / (|g| + eps)
    th1, _, _ = mlp.adam_step(theta, g, m, v, 1, lr=1e-3)
    assert np.allclose(theta - th1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    for step in range(1, 301):
        _, g = mlp.loss_and_grad(theta, X, t)
        theta, m, v = mlp.adam_step(theta, g, m, v, step, lr=1e-2)
    l1, _ = mlp.loss_and_grad(theta, X, t)
    assert l1 < 0.1 * l0


def test_capacity_rule():
    r = np.array([0.0, 3.0, 10.0, 30.0])
    cap = mlp.capacity(np.log1p(r))
    assert list(cap) == [4, 8, 16, 40]
