"""The library's gCQ contour (gcq_contour, host code) against the oracle's
points and weights, its Cauchy property where the oracle loses digits (step
ratios near 1), its symmetry and its argument errors.  CPU only."""
import numpy as np
import pytest

import paper_2505_00715_amd as g
from oracle import contour as C


@pytest.mark.parametrize("q", [1.2, 1.5, 4.0, 20.0, 1000.0])
@pytest.mark.parametrize("n_q", [1, 7, 32, 65])
def test_contour_matches_oracle(q, n_q):
    s, w = g.contour(n_q, 0.01, q * 0.01)
    so, wo = C.contour(n_q, 0.01, q * 0.01)
    assert np.max(np.abs(s - so) / np.abs(so)) <= 1e-11
    assert np.max(np.abs(w - wo) / np.abs(wo)) <= 1e-11


@pytest.mark.parametrize("q", [1.001, 1.01, 3.0, 1e6])
def test_contour_cauchy_and_symmetry(q):
    dt = 0.02
    s, w = g.contour(65, dt, q * dt, 1.0)
    assert np.all(s.real > 0)
    assert np.max(np.abs(s - np.conj(s[::-1]))) <= 1e-13 * np.max(np.abs(s))
    assert abs(s[32].imag) <= 1e-13 * abs(s[32])        # odd count: the middle point is real
    tol = 1e-12 if q < 1e5 else 1e-8
    for z in (1.0 / (q * dt), 1.0 / dt):
        assert abs(np.sum(w / (s - z)) + 1.0) < tol     # clockwise: -1 inside
    assert abs(np.sum(w / (s + 10.0 / dt))) < tol       # 0 outside


def test_stage_ratio_scales_q():
    a = g.contour(16, 0.01, 0.02, 5.0)
    b = g.contour(16, 0.01, 0.1, 1.0)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-14)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-14)


def test_contour_argument_errors():
    for args in ((0, 0.01, 0.02, 1.0), (8, 0.0, 0.02, 1.0), (8, 0.02, 0.01, 1.0),
                 (8, 0.01, 0.02, 0.5), (8, 0.01, 0.01, 1.0)):
        with pytest.raises(g.GcqError):
            g.contour(*args)


def _cube_rows():
    import os
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "cube_refinement.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _cube_rows(), ids=lambda r: f"level{int(r[0])}")
def test_contour_points_match_cube_table(row):
    """N_Q of the unit-cube table (Sec. 5.1, 2-stage Radau IIA) is the half of
    N (ln N)^2 points: the oracle's rule and the library's both give it."""
    N, half = int(row[5]), int(row[6])
    assert C.n_points(N, 2) == 2 * half
    assert g.contour_points(N, 2) == 2 * half


def test_contour_points_one_stage_and_errors():
    for N in (2, 10, 64, 1000, 12345):
        assert g.contour_points(N, 1) == C.n_points(N, 1)
        assert g.contour_points(N, 3) == C.n_points(N, 3)
    assert C.n_points(100, 1) == 2 * round(100 * np.log(100) / 2)
    for bad in ((1, 1), (0, 2), (10, 0)):
        with pytest.raises(g.GcqError):
            g.contour_points(*bad)
        with pytest.raises(ValueError):
            C.n_points(*bad)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_contour_steps_match_oracle(m):
    from oracle import gcq as G
    A = G.radau_iia(m)
    got = g.contour_steps(A, 0.01, 0.035)
    ref = G.contour_steps(A, 0.01, 0.035)
    np.testing.assert_allclose(got, ref, rtol=1e-10)


def test_contour_steps_errors():
    with pytest.raises(g.GcqError):
        g.contour_steps(np.zeros((2, 2)), 0.01, 0.02)          # singular
    with pytest.raises(g.GcqError):
        g.contour_steps(np.eye(5), 0.01, 0.02)                 # m > 4
    with pytest.raises(g.GcqError):
        g.contour_steps(np.array([[1.0]]), 0.02, 0.01)         # dt_max < dt_min
    with pytest.raises(g.GcqError):
        g.contour_steps(np.array([[-1.0, 0.0], [0.0, -2.0]]), 0.01, 0.02)   # no growth interval
