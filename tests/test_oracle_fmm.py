"""Pins of the FMM-based 3D-ACA oracle (Sec. 4, eq. cheb; Alg. 1) against
what mathematics fixes: polynomial reproduction and the Chebyshev remainder
of the interpolation, the exact nesting of son and parent interpolation, the
interpolated far blocks against the independently evaluated dense entries
(geometric convergence in the order), and the compressed product against the
dense product."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev

from oracle import entries, fmm, freqmap
from oracle.geometry import Panels
from oracle.tree import ClusterTree, block_tree
from synth import freq, mesh, rhs


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_lagrange_basis_at_chebyshev_nodes(p):
    t = fmm.cheb_nodes(p)
    # the nodes are the zeros of T_p
    assert np.allclose(chebyshev.chebval(t, [0] * p + [1]), 0.0, atol=1e-13)
    Lb = fmm.lagrange_1d(t, p)
    assert np.allclose(Lb, np.eye(p), atol=1e-13)
    x = np.linspace(-1, 1, 41)
    assert np.allclose(fmm.lagrange_1d(x, p).sum(axis=1), 1.0, atol=1e-13)


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_chebyshev_remainder_of_the_monomial(p):
    """Interpolating t^a (a < p) is exact; for t^p the remainder is
    2^(1-p) T_p(t), the monic Chebyshev polynomial (it vanishes at the nodes
    and t^p - 2^(1-p) T_p has degree p - 1)."""
    x = np.linspace(-1.2, 1.2, 57)
    Lx = fmm.lagrange_1d(x, p)
    t = fmm.cheb_nodes(p)
    for a in range(p):
        assert np.allclose(Lx @ t ** a, x ** a, atol=1e-12)
    rem = x ** p - Lx @ t ** p
    Tp = chebyshev.chebval(x, [0] * p + [1])
    assert np.allclose(rem, 2.0 ** (1 - p) * Tp, atol=1e-12)


def test_tensor_interpolation_reproduces_polynomials():
    rng = np.random.default_rng(0)
    p = 4
    box = (np.array([0.3, -1.0, 2.0]), np.array([0.5, 0.25, 1.5]))
    coef = rng.standard_normal((p, p, p))

    def poly(pts):
        u = (pts - box[0]) / box[1]
        out = np.zeros(len(pts))
        for a in range(p):
            for b in range(p):
                for c in range(p):
                    out += coef[a, b, c] * u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** c
        return out

    pts = box[0] + box[1] * rng.uniform(-1, 1, (50, 3))
    S = fmm.interp(box, pts, p)
    vals = poly(fmm.box_nodes(box, p))
    assert np.allclose(S @ vals, poly(pts), atol=1e-11)
    # node numbering n = a_x + p a_y + p^2 a_z
    nodes = fmm.box_nodes(box, p)
    t = fmm.cheb_nodes(p)
    assert np.allclose(nodes[1 + p * 2 + p * p * 3], box[0] + box[1] * t[[1, 2, 3]])


@pytest.fixture(scope="module")
def sphere():
    xyz, tri = mesh.icosphere(2)
    P = Panels(xyz, tri)
    T = ClusterTree(P, 16)
    B = block_tree(T, 1.0)
    return P, T, B


def test_son_interpolation_nests_in_the_parent(sphere):
    """R_P = [R_s0 T_s0; R_s1 T_s1] and L_P likewise, exactly (the parent's
    Lagrange polynomials have degree p - 1 in each coordinate)."""
    P, T, B = sphere
    p = 4
    for c in range(len(T.begin)):
        if T.is_leaf(c):
            continue
        bp = fmm.box_of(T, c)
        Rp = fmm.r_op(P, bp, T.indices(c), p)
        Lp = fmm.l_op(P, bp, T.indices(c), p)
        parts_R, parts_L = [], []
        for s in (T.son0[c], T.son1[c]):
            bs = fmm.box_of(T, int(s))
            Ts = fmm.transfer(bs, bp, p)
            parts_R.append(fmm.r_op(P, bs, T.indices(int(s)), p) @ Ts)
            parts_L.append(fmm.l_op(P, bs, T.indices(int(s)), p) @ Ts)
        scale = np.abs(Rp).max()
        assert np.abs(np.vstack(parts_R) - Rp).max() <= 1e-12 * scale
        assert np.abs(np.vstack(parts_L) - Lp).max() <= 1e-12


def test_far_blocks_converge_to_the_dense_entries(sphere):
    """The interpolated far blocks against entries.block (the far rule
    evaluated directly): the error falls geometrically with the order."""
    P, T, B = sphere
    s = np.array([0.5 + 0.3j, 4.0 + 8.0j])
    far = [(X, Y) for X, Y, adm in B if adm]
    rng = np.random.default_rng(1)
    pick = [far[i] for i in rng.choice(len(far), 6, replace=False)]
    errs = []
    for p in (2, 4, 6, 8):
        num = den = 0.0
        for X, Y in pick:
            A = entries.block(P, T.indices(X), T.indices(Y), s, 1.0)
            Af = fmm.far_block_dense(P, T, X, Y, s, 1.0, p)
            num += np.linalg.norm(Af - A) ** 2
            den += np.linalg.norm(A) ** 2
        errs.append(np.sqrt(num / den))
    assert all(e2 < 0.5 * e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4, errs


def test_m2l_3d_aca_and_product_against_dense(sphere):
    """Alg. 1 on the M2L tensors holds the frequency tolerance on each far
    block's operator; the compressed product of all blocks against the dense
    product at every frequency, within the interpolation error plus the
    tolerances."""
    P, T, B = sphere
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    rep, conj = freqmap.representatives(s)
    K = freqmap.distinct(rep)
    kpos = {int(k): i for i, k in enumerate(K)}
    p, tol = 6, 1e-6
    blocks = fmm.fmm3d(P, T, B, s[K], 1.0, p, tol, 40)
    far = [b for b in blocks if isinstance(b, fmm.FmmBlock)]
    assert len(far) > 0
    for Bk, (X, Y, adm) in zip(blocks, B):
        if not adm:
            continue
        M = fmm.m2l(fmm.box_of(T, X), fmm.box_of(T, Y), s[K], 1.0, p)
        approx = sum(Bk.b3.fibers[d][:, None, None] * Bk.b3.slices[d][None] for d in range(Bk.rank))
        assert np.linalg.norm(approx - M) <= 20 * tol * np.linalg.norm(M)
    X = rhs.random_complex(len(s), P.n, 0)
    Y = fmm.product(blocks, X, rep, conj, kpos)
    A = entries.dense(P, s, 1.0)
    Yd = np.einsum("kij,kj->ki", A, X)
    per_k = np.linalg.norm(Y - Yd, axis=1) / np.linalg.norm(Yd, axis=1)
    assert per_k.max() < 1e-4, per_k.max()
