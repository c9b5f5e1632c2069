"""Pins of the double-layer oracle (oracle.dlp; Sec. 2, eq. dlp, transformed as
in Sec. 3): the kernel's normal derivative against a finite difference of the
single-layer kernel, the collocation matrix's row sums on spheres against the
closed form of the double layer of a constant density (Gauss's solid-angle
identity -1/2 as s -> 0), with the discretisation error falling under
refinement, and the tiers."""
import numpy as np
import pytest

from oracle import dlp, entries
from oracle.geometry import Panels
from synth import mesh

S = np.array([1e-6, 1.0, 3.0 + 2.0j, 10.0 - 5.0j])


def test_kernel_is_the_normal_derivative_of_the_single_layer_kernel():
    rng = np.random.default_rng(3)
    for s in (0.5, 2.0 + 3.0j, 7.0 - 1.0j):
        x = rng.standard_normal(3)
        y = rng.standard_normal(3)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        h = 1e-5
        up = entries.kernel(np.linalg.norm(x - (y + h * n)), s, 1.5)
        um = entries.kernel(np.linalg.norm(x - (y - h * n)), s, 1.5)
        fd = (up - um) / (2 * h)
        an = dlp.kernel_dn(x - y, n, s, 1.5)
        assert abs(an - fd) <= 1e-8 * abs(an)


def test_sphere_closed_form_limits():
    assert abs(dlp.sphere_constant(1.0, 1e-9, 1.0) + 0.5) < 1e-8
    # large kappa R: only the neighbourhood contributes, -1/(2 kappa R)
    assert abs(dlp.sphere_constant(2.0, 1e4, 1.0) * 4e4 + 1.0) < 1e-12
    # against direct quadrature of -(1/4R) int_0^{2R} (1 + k r) exp(-k r) dr
    from scipy import integrate
    R, s = 0.7, 3.0 + 2.0j
    re = integrate.quad(lambda r: ((1 + s * r) * np.exp(-s * r)).real, 0, 2 * R, epsabs=1e-14)[0]
    im = integrate.quad(lambda r: ((1 + s * r) * np.exp(-s * r)).imag, 0, 2 * R, epsabs=1e-14)[0]
    assert abs(dlp.sphere_constant(R, s, 1.0) + (re + 1j * im) / (4 * R)) < 1e-13


@pytest.fixture(scope="module")
def spheres():
    out = []
    for sub in (1, 2):
        xyz, tri = mesh.icosphere(sub)
        P = Panels(xyz, tri)
        out.append((P, dlp.dense(P, S, 1.0)))
    return out


def test_row_sums_match_the_sphere_closed_form(spheres):
    exact = dlp.sphere_constant(1.0, S, 1.0)
    errs = []
    for P, K in spheres:
        errs.append(np.max(np.abs(K.sum(-1) - exact[:, None]), axis=1))
    assert errs[0][0] < 1e-5 and errs[1][0] < 1e-5        # Gauss: -1/2 on a closed polyhedron
    assert np.all(errs[1] < 2e-2)
    assert np.all(errs[1][1:3] < errs[0][1:3] / 2.5)         # converging under refinement
    assert errs[1][3] < errs[0][3]


def test_tiers(spheres):
    P, K = spheres[1]
    assert np.all(np.diagonal(K, axis1=1, axis2=2) == 0)   # flat panel: d . n_y = 0
    # a far pair is the 7-point rule, a near pair the 112-point rule
    i = 0
    d2 = ((P.centroid - P.centroid[i]) ** 2).sum(1)
    jf = int(np.argmax(d2))
    jn = int(np.nonzero((d2 < 4 * P.h2) & (np.arange(P.n) != i))[0][0])
    assert entries.tier(P, i, jf) == entries.FAR and entries.tier(P, i, jn) == entries.NEAR
    for j, (pts, wts) in ((jf, (P.qp[jf], P.qw[jf])), (jn, P.near_rule(jn))):
        ref = [np.sum(dlp.kernel_dn(P.centroid[i] - pts, P.normal[j], s, 1.0) * wts) for s in S]
        np.testing.assert_allclose(K[:, i, j], ref, rtol=1e-13)
    # the normal derivative points along the outward normal: on a convex
    # surface every off-diagonal entry at small s is negative
    assert np.all(K[1].real[~np.eye(P.n, dtype=bool)] < 0)
