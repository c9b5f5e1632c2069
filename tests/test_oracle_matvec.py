"""Pins of the oracle's products: the per-frequency H-matrix and compressed
products equal the dense product with the reconstructed approximant, conjugate
representatives give the same result as direct evaluation, and the eq. product
regrouping equals the sum of the per-frequency columns."""
import numpy as np

from oracle import aca, aca3d, entries, freqmap, matvec
from oracle.geometry import Panels
from oracle.tree import ClusterTree, block_tree
from synth import freq, mesh, rhs


def _setup():
    xyz, tri = mesh.icosphere(2)
    P = Panels(xyz, tri)
    T = ClusterTree(P, 16)
    blocks = block_tree(T, 1.0)
    s = freq.bdf2_circle(8, 0.05, 1e-8 ** (1 / 8))
    return P, T, blocks, s


def test_dense_matches_numpy():
    P, T, blocks, s = _setup()
    A = entries.dense(P, s, 1.0)
    X = rhs.random_complex(len(s), P.n, 0)
    Y = matvec.dense(A, X)
    for k in range(len(s)):
        assert np.allclose(Y[k], A[k] @ X[k], rtol=1e-14, atol=0)


def test_hmatrix_equals_reconstruction_and_conjugate_rule():
    P, T, blocks, s = _setup()
    rep, conj = freqmap.representatives(s)
    assert conj.sum() == 3 and (rep[5:] == [3, 2, 1]).all()
    X = rhs.random_complex(len(s), P.n, 0)
    hb = []
    recon = np.zeros((len(s), P.n, P.n), dtype=complex)
    for a, b, adm in blocks:
        I, J = T.indices(a), T.indices(b)
        data = {}
        for k in freqmap.distinct(rep):
            if adm:
                U, V, _ = aca.aca_block(P, I, J, s[k], 1.0, 1e-8, 1000)
                data[k] = (U, V)
                recon[k][np.ix_(I, J)] = U @ V.conj().T
            else:
                data[k] = entries.block(P, I, J, [s[k]], 1.0)[0]
                recon[k][np.ix_(I, J)] = data[k]
        hb.append((I, J, adm, data))
    for k in range(len(s)):
        if conj[k]:
            recon[k] = np.conj(recon[rep[k]])
    Y = matvec.hmatrix(hb, X, rep, conj)
    Yd = matvec.dense(recon, X)
    assert np.abs(Y - Yd).max() <= 1e-13 * np.abs(Yd).max()
    # and the approximation is close to the true dense operator at every k
    Ad = entries.dense(P, s, 1.0)
    Yt = matvec.dense(Ad, X)
    assert np.linalg.norm(Y - Yt) <= 1e-6 * np.linalg.norm(Yt)


def test_compressed_product_identities():
    P, T, blocks, s = _setup()
    rep, conj = freqmap.representatives(s)
    K = freqmap.distinct(rep)
    kpos = {int(k): p for p, k in enumerate(K)}
    b3 = [aca3d.aca3d_mesh_block(P, T.indices(a), T.indices(b), s[K], 1.0, adm, 1e-8, 1e-7, 40)
          for a, b, adm in blocks]
    X = rhs.random_complex(len(s), P.n, 1)
    Y = matvec.compressed(b3, X, rep, conj, kpos)
    # reconstruction of the whole 3D approximant
    recon = np.zeros((len(s), P.n, P.n), dtype=complex)
    for B in b3:
        Tt = B.tensor()
        for k in range(len(s)):
            blk = Tt[kpos[rep[k]]]
            recon[k][np.ix_(B.rows, B.cols)] = np.conj(blk) if conj[k] else blk
    Yd = matvec.dense(recon, X)
    assert np.abs(Y - Yd).max() <= 1e-12 * np.abs(Yd).max()
    # regrouping of eq. product == sum of the per-frequency columns
    y = matvec.weighted_sum(b3, X, rep, conj, kpos)
    assert np.abs(y - Y.sum(0)).max() <= 1e-12 * np.abs(y).max()
    # close to the true operator
    Ad = entries.dense(P, s, 1.0)
    Yt = matvec.dense(Ad, X)
    assert np.linalg.norm(Y - Yt) <= 1e-5 * np.linalg.norm(Yt)
