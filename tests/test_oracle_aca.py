"""Pins of the oracle's ACA and recompression: exact recovery of low-rank
blocks, exactness at zero tolerance, error bounds on real far blocks against
the dense block, the truncated-SVD lower bound on the rank, the recursive norm
against the direct Frobenius norm, and recompression against LAPACK's SVD of
the product."""
import numpy as np
import pytest

from oracle import aca, entries
from oracle.geometry import Panels
from oracle.tree import ClusterTree, block_tree
from synth import mesh


def _fns(A):
    return (lambda i: A[i, :].copy()), (lambda j: A[:, j].copy())


@pytest.mark.parametrize("m,n,k", [(30, 40, 1), (50, 20, 3), (64, 64, 7)])
def test_exact_low_rank_recovered(m, n, k):
    rng = np.random.default_rng(k)
    A = (rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))) @ \
        (rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n)))
    U, V, info = aca.aca(*_fns(A), m, n, 1e-10, 1000)
    # after k terms the residual is zero up to rounding; the stopping test then
    # accepts (and keeps) one more term of rounding size at most
    assert info["rank"] in (k, k + 1)
    assert np.linalg.norm(A - U @ V.conj().T) <= 1e-12 * np.linalg.norm(A)
    Ub, Vb, _, _ = aca.recompress(U, V, 1e-10)
    assert Ub.shape[1] == k


def test_zero_tolerance_full_rank_is_exact():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((12, 9)) + 1j * rng.standard_normal((12, 9))
    U, V, info = aca.aca(*_fns(A), 12, 9, 0.0, 1000)
    assert info["rank"] == 9
    assert np.linalg.norm(A - U @ V.conj().T) <= 1e-12 * np.linalg.norm(A)


def test_zero_block_and_zero_rows():
    A = np.zeros((10, 8), dtype=complex)
    U, V, info = aca.aca(*_fns(A), 10, 8, 1e-5, 100)
    assert info["rank"] == 0 and U.shape == (10, 0)
    B = np.zeros((10, 8), dtype=complex)
    B[7, :] = np.arange(1, 9)             # only row 7 is non-zero: reached by the fallback
    U, V, info = aca.aca(*_fns(B), 10, 8, 1e-5, 100)
    assert info["rank"] == 1 and np.allclose(U @ V.conj().T, B)


def test_max_rank_cap_reported():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((20, 20)) + 0j
    U, V, info = aca.aca(*_fns(A), 20, 20, 1e-10, 5)
    assert info["rank"] == 5 and info["capped"]


def _far_blocks(sub, leaf):
    xyz, tri = mesh.icosphere(sub)
    P = Panels(xyz, tri)
    T = ClusterTree(P, leaf)
    return P, T, [(a, b) for a, b, adm in block_tree(T, 1.0) if adm]


@pytest.mark.parametrize("s", [1.0, 26.67 + 0j, 60.0 + 40.0j])
def test_far_blocks_error_rank_and_norm(s):
    P, T, far = _far_blocks(3, 32)
    assert len(far) > 10
    tol = 1e-5
    ratios = []
    for a, b in far[:: max(1, len(far) // 40)]:
        I, J = T.indices(a), T.indices(b)
        A = entries.block(P, I, J, [s], 1.0)[0]
        U, V, info = aca.aca_block(P, I, J, s, 1.0, tol, 1000)
        S = U @ V.conj().T
        nA = np.linalg.norm(A)
        # the stopping test estimates the error from the last term only: the
        # true block error stays within a modest factor of eps (<= 16 eps was
        # the worst over all 1852 far blocks of this mesh at three frequencies)
        ratios.append(np.linalg.norm(A - S) / (tol * nA))
        # recursive norm of eq.-norm type equals the direct Frobenius norm
        assert abs(np.sqrt(info["norm2"]) - np.linalg.norm(S)) <= 1e-10 * np.linalg.norm(S)
        # no rank-r approximation can beat the truncated SVD: the ACA rank is at
        # least the SVD rank that reaches the ACA's achieved error
        sv = np.linalg.svd(A, compute_uv=False)
        err = np.linalg.norm(A - S)
        tail = np.sqrt(np.concatenate([np.cumsum((sv ** 2)[::-1])[::-1], [0.0]]))
        r_svd = int(np.nonzero(tail <= err * (1 + 1e-9))[0][0])
        assert info["rank"] >= r_svd
    assert max(ratios) <= 20.0 and np.mean(ratios) <= 1.0


def test_recompression_matches_svd_of_product():
    rng = np.random.default_rng(2)
    m, n, k = 40, 30, 9
    # factors with geometrically decaying columns
    U = (rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))) * (0.1 ** np.arange(k))
    V = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    sv = np.linalg.svd(U @ V.conj().T, compute_uv=False)
    for tol in [0.0, 1e-3, 1e-6]:
        Ub, Vb, s_kept, s_all = aca.recompress(U, V, tol)
        assert np.allclose(s_all, sv[:k], rtol=1e-12, atol=1e-14 * sv[0])
        t = Ub.shape[1]
        # output is the truncated SVD: its singular values are the leading ones
        sv_out = np.linalg.svd(Ub @ Vb.conj().T, compute_uv=False)[:t]
        assert np.allclose(sv_out, sv[:t], rtol=1e-10)
        # Vb has orthonormal columns
        assert np.allclose(Vb.conj().T @ Vb, np.eye(t), atol=1e-12)
        # truncation rule: smallest t with tail <= tol * total
        tail = np.sqrt((sv[t:k] ** 2).sum())
        assert tail <= tol * np.sqrt((sv[:k] ** 2).sum()) + 1e-15 * sv[0]
        if t > 0:
            assert np.sqrt((sv[t - 1:k] ** 2).sum()) > tol * np.sqrt((sv[:k] ** 2).sum())
    Ub, Vb, _, _ = aca.recompress(U, V, 0.0)
    assert np.linalg.norm(U @ V.conj().T - Ub @ Vb.conj().T) <= 1e-12 * np.linalg.norm(U @ V.conj().T)
