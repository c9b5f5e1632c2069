"""Points and weights of the gCQ integration contour (oracle; App. A).

Test infrastructure: imported only by the tests, the smoke check and the
benchmark's CPU baseline.  Plain float64 numpy/scipy, written from the
appendix's formulas.

Reading used (App. A; parts of the printed formulas are garbled):

  q       = ratio of the largest to the smallest step size, times
            `stage_ratio` (5 max|lambda_i(A)| / min|lambda_i(A)| for a
            Runge-Kutta method of more than one stage, 1 for implicit Euler)
  k       = (q - sqrt(2q - 1)) / (q + sqrt(2q - 1))        elliptic modulus
  K, K'   = K(k^2), K(1 - k^2): complete elliptic integrals of the first kind,
            written with the parameter m = k^2 (the complementary integral
            takes 1 - m)
  sigma_l = -K + (l - 1/2) 4K / N_Q + i K' / 2,   l = 1 .. N_Q
  gamma   = ( sqrt(2q-1) (1/k + sn) / (1/k - sn) - 1 ) / (dt_min (q - 1))
  gamma'  = sqrt(2q-1) / (dt_min (q - 1)) * 2 cn dn / (k (1/k - sn)^2)
  s_l     = gamma(sigma_l)
  w_l     = 4K / (2 pi i N_Q) * gamma'(sigma_l)

with sn, cn, dn the Jacobi elliptic functions of modulus k.  The printed
weight shows only "4K(k^2) / (1 pi i)"; the reading takes the trapezoidal
rule with step 4K/N_Q over one real period for (1 / 2 pi i) times the contour
integral, which the tests check through Cauchy's integral formula.  The
number of points N_Q (N log N for N steps in the paper) is the caller's.
q = 1 (constant steps, k = 0) is excluded, as the appendix notes; a caller
with constant steps perturbs q slightly above 1.

Near q = 1 (k and m tiny) the imaginary-part functions, of parameter 1 - m,
lose digits here because scipy takes the parameter rather than its
complement: about 1e-10 relative at q = 1.01.

Jacobi functions of the complex argument x + iy follow from those of real
argument (modulus k at x, complementary modulus at y) by the addition
formulas (Abramowitz & Stegun 16.21.2-4); scipy's real-argument routines
serve as that step.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def n_points(n_steps: int, stages: int) -> int:
    """Number N_Q of contour points for N = n_steps steps (Sec. 3, cost estimate
    after eq. gcq_formula, and App. A): N log N for one stage, N (log N)^2 for
    m > 1 stages, natural logarithm.  Reading: the points come in conjugate
    pairs and only half of them are computed (Sec. 5.1), so N_Q is taken as
    twice the rounded half, 2 round(N (log N)^p / 2); the half N_Q / 2 is what
    the table of the unit-cube meshes (Sec. 5.1) lists for 2-stage Radau IIA."""
    if n_steps < 2 or stages < 1:
        raise ValueError("need n_steps >= 2 and stages >= 1")
    p = 1 if stages == 1 else 2
    return 2 * int(round(n_steps * np.log(n_steps) ** p / 2.0))


def modulus(q: float) -> float:
    r = np.sqrt(2.0 * q - 1.0)
    return (q - r) / (q + r)


def jacobi_complex(x, y, m):
    """sn, cn, dn of x + i y with parameter m (x, y real arrays)."""
    s, c, d, _ = special.ellipj(x, m)
    s1, c1, d1, _ = special.ellipj(y, 1.0 - m)
    den = c1 ** 2 + m * s ** 2 * s1 ** 2
    sn = (s * d1 + 1j * c * d * s1 * c1) / den
    cn = (c * c1 - 1j * s * d * s1 * d1) / den
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / den
    return sn, cn, dn


def contour(n_q: int, dt_min: float, dt_max: float, stage_ratio: float = 1.0):
    """Points s (n_q,) and weights w (n_q,) of the contour quadrature."""
    q = stage_ratio * dt_max / dt_min
    if not q > 1.0:
        raise ValueError("q must exceed 1")
    k = modulus(q)
    m = k * k
    K = special.ellipk(m)
    Kp = special.ellipkm1(m)   # K(1 - m) without forming 1 - m
    l = np.arange(1, n_q + 1)
    x = -K + (l - 0.5) * 4.0 * K / n_q
    y = np.full(n_q, 0.5 * Kp)
    sn, cn, dn = jacobi_complex(x, y, m)
    r = np.sqrt(2.0 * q - 1.0)
    scale = 1.0 / (dt_min * (q - 1.0))
    gamma = scale * (r * (1.0 / k + sn) / (1.0 / k - sn) - 1.0)
    dgamma = scale * r * 2.0 * cn * dn / (k * (1.0 / k - sn) ** 2)
    w = 4.0 * K / (2j * np.pi * n_q) * dgamma
    return gamma, w


def gamma_of(sigma, dt_min: float, q: float):
    """gamma(sigma) at complex sigma (for derivative checks)."""
    k = modulus(q)
    sn, _, _ = jacobi_complex(np.real(sigma), np.imag(sigma), k * k)
    r = np.sqrt(2.0 * q - 1.0)
    return (r * (1.0 / k + sn) / (1.0 / k - sn) - 1.0) / (dt_min * (q - 1.0))
