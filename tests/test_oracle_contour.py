"""Pins of the contour oracle (App. A): the complete elliptic integrals against
their defining integrals, the complex Jacobi functions against their
identities, quasi-periods and derivative, gamma' against the derivative of
gamma, the conjugate symmetry of points and weights, and the weights against
Cauchy's integral formula."""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import contour as C


@pytest.mark.parametrize("q", [1.05, 2.0, 20.0])
def test_complete_integrals_against_definition(q):
    k = C.modulus(q)
    assert 0.0 < k < 1.0
    m = k * k
    for par in (m, 1.0 - m):
        # the definition with x = sin(theta), which removes the end-point singularity
        val, _ = integrate.quad(lambda t: 1.0 / np.sqrt(1.0 - par * np.sin(t) ** 2), 0.0, np.pi / 2,
                                epsabs=0.0, epsrel=1e-13, limit=400)
        assert abs(special.ellipk(par) - val) <= 1e-10 * val


@pytest.mark.parametrize("m", [0.01, 0.3, 0.9])
def test_complex_jacobi_functions(m):
    rng = np.random.default_rng(3)
    K, Kp = special.ellipk(m), special.ellipk(1.0 - m)
    x = rng.uniform(-K, 3 * K, 40)
    y = rng.uniform(-0.9 * Kp, 0.9 * Kp, 40)
    sn, cn, dn = C.jacobi_complex(x, y, m)
    assert np.max(np.abs(sn ** 2 + cn ** 2 - 1.0)) < 1e-12
    assert np.max(np.abs(dn ** 2 + m * sn ** 2 - 1.0)) < 1e-12
    # periods 4K (real) and 2iK' (imaginary) of sn
    sn4, _, _ = C.jacobi_complex(x + 4 * K, y, m)
    sn2, _, _ = C.jacobi_complex(x, y + 2 * Kp, m)
    assert np.max(np.abs(sn4 - sn)) < 1e-10
    assert np.max(np.abs(sn2 - sn)) < 1e-9
    # d sn / du = cn dn, along the real and the imaginary direction
    h = 1e-6
    for dx, dy, f in ((h, 0.0, 1.0), (0.0, h, 1j)):
        sp, _, _ = C.jacobi_complex(x + dx, y + dy, m)
        sm, _, _ = C.jacobi_complex(x - dx, y - dy, m)
        fd = (sp - sm) / (2 * h * f)
        assert np.max(np.abs(fd - cn * dn) / np.maximum(1.0, np.abs(cn * dn))) < 1e-6
    # sn(K) = 1 on the real axis
    s1, _, _ = C.jacobi_complex(np.array([K]), np.array([0.0]), m)
    assert abs(s1[0] - 1.0) < 1e-12


def test_gamma_prime_is_the_derivative_of_gamma():
    dt_min, q = 0.01, 6.0
    k = C.modulus(q)
    K, Kp = special.ellipk(k * k), special.ellipk(1 - k * k)
    n_q = 24
    s, w = C.contour(n_q, dt_min, q * dt_min)
    sig = -K + (np.arange(1, n_q + 1) - 0.5) * 4 * K / n_q + 0.5j * Kp
    assert np.max(np.abs(C.gamma_of(sig, dt_min, q) - s)) <= 1e-12 * np.max(np.abs(s))
    h = 1e-6
    fd = (C.gamma_of(sig + h, dt_min, q) - C.gamma_of(sig - h, dt_min, q)) / (2 * h)
    dgamma = w * (2j * np.pi * n_q) / (4 * K)
    assert np.max(np.abs(fd - dgamma)) <= 1e-6 * np.max(np.abs(dgamma))


@pytest.mark.parametrize("q", [1.5, 4.0, 20.0])
def test_points_and_weights_conjugate_symmetric(q):
    s, w = C.contour(32, 0.01, q * 0.01)
    assert np.max(np.abs(s - np.conj(s[::-1]))) <= 1e-13 * np.max(np.abs(s))
    assert np.max(np.abs(w - np.conj(w[::-1]))) <= 1e-13 * np.max(np.abs(w))
    assert np.all(s.real > 0)


@pytest.mark.parametrize("q", [1.5, 4.0, 20.0])
def test_weights_reproduce_cauchys_formula(q):
    """sum_l w_l / (s_l - z): -1 for z inside the contour (it is traversed
    clockwise as Re sigma grows), 0 outside; inside lie the reciprocal step
    sizes [1/dt_max, 1/dt_min]."""
    dt_min = 0.01
    s, w = C.contour(64, dt_min, q * dt_min)
    for z in (1.0 / (q * dt_min), 1.0 / (np.sqrt(q) * dt_min), 1.0 / dt_min):
        assert abs(np.sum(w / (s - z)) + 1.0) < 1e-8
    for z in (-5.0 / dt_min, 10.0 / dt_min, 3j / dt_min):
        assert abs(np.sum(w / (s - z))) < 1e-8
    # an entire function integrates to zero
    assert abs(np.sum(w * np.exp(-s * dt_min))) < 1e-8


def test_constant_steps_are_rejected():
    with pytest.raises(ValueError):
        C.contour(16, 0.01, 0.01)


@pytest.mark.parametrize("q", [1.5, 4.0, 20.0])
def test_contour_passes_through_zero_and_two_over_dt_min(q):
    """gamma(-K + i K'/2) = 0 and gamma(K + i K'/2) = 2 / dt_min (sn = -+1/sqrt(k) there)."""
    dt_min = 0.01
    k = C.modulus(q)
    K, Kp = special.ellipk(k * k), special.ellipkm1(k * k)
    g = C.gamma_of(np.array([-K + 0.5j * Kp, K + 0.5j * Kp]), dt_min, q)
    assert abs(g[0]) <= 1e-10 / dt_min
    assert abs(g[1] - 2.0 / dt_min) <= 1e-10 / dt_min
