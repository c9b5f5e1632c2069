"""Complex frequency sets (input data only).

The gCQ discretisation needs the Laplace-domain operator at a set of complex
points s_l (Sec. 3, temporal discretisation; App. A).  For the synthetic
workloads the points come from the BDF2 generating function on a circle of
radius lam < 1, the constant-step special case of the contour quadrature:

    s_k = delta(lam * exp(2 pi i k / L)) / dt,   delta(z) = (1 - z) + (1 - z)^2 / 2,

k = 0..L-1.  The set is closed under conjugation (s_{L-k} = conj(s_k)); s_0 and
s_{L/2} are real.  The library accepts any set of points with Re s > 0.
"""
from __future__ import annotations

import numpy as np


def bdf2_circle(L: int, dt: float, lam: float) -> np.ndarray:
    k = np.arange(L)
    z = lam * np.exp(2j * np.pi * k / L)
    s = ((1.0 - z) + 0.5 * (1.0 - z) ** 2) / dt
    # make the conjugate pairing exact in floating point
    for kk in range(1, (L + 1) // 2):
        s[L - kk] = np.conj(s[kk])
    if L % 2 == 0:
        s[L // 2] = s[L // 2].real
    s[0] = s[0].real
    return s.astype(np.complex128)


def steps_contour(n_steps: int, dt: float):
    """L = 2N points with radius lam = 10**(-8/N): the rule the 64- and
    256-point workloads use (N = 32, 128)."""
    L = 2 * n_steps
    lam = 10.0 ** (-8.0 / n_steps)
    return bdf2_circle(L, dt, lam)
