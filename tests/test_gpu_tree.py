"""gcq_upload_cluster_tree on the GPU: the oracle's partition injected into a
context gives bit-identical 3D-ACA factors and products to the library's own
build of the same partition; a partition the library does not build (a PCA
split, as the paper's cluster tree of Sec. 4 uses) gives a product that matches
the dense oracle."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import entries, matvec
from oracle.geometry import Panels
from synth import freq, mesh, rhs
from tests._gpu_common import from_dev, rel, to_dev
from tests._oracle_tree_blocks import oracle_tree, tree_arrays

pytestmark = pytest.mark.gpu


def _ctx(xyz, tri, s):
    ctx = g.Context(0)
    ctx.upload_mesh(xyz, tri, 1.0)
    ctx.set_frequencies(s, True)
    return ctx


@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_uploaded_tree_gives_bit_identical_factors(prec):
    xyz, tri = mesh.icosphere(3)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    P, T, B, _, _ = oracle_tree(xyz, tri, 32, 1.0)
    a = _ctx(xyz, tri, s)
    a.build_cluster_tree(32, 1.0)
    b = _ctx(xyz, tri, s)
    b.upload_cluster_tree(*tree_arrays(T, B))
    sa = a.aca3d(1e-6, 1e-5, 40, prec)
    sb = b.aca3d(1e-6, 1e-5, 40, prec)
    assert sa.storage_bytes == sb.storage_bytes and sa.slice_rank_sum == sb.slice_rank_sum
    nK = len(s) // 2 + 1
    for blk in range(len(B)):
        fa, ca, la = a.get_aca3d_block(blk, nK)
        fb, cb, lb = b.get_aca3d_block(blk, nK)
        assert np.array_equal(fa, fb) and np.array_equal(ca, cb) and np.array_equal(la, lb)
    X = to_dev(rhs.random_complex(len(s), P.n, 0), prec).reshape(-1)
    Ya, Yb = torch.zeros_like(X), torch.zeros_like(X)
    a.compressed_matvec(g.PER_FREQUENCY, prec, X, Ya)
    b.compressed_matvec(g.PER_FREQUENCY, prec, X, Yb)
    # same factors; the product's float atomics may sum in another order
    assert rel(from_dev(Yb), from_dev(Ya)) <= (1e-14 if prec == g.C128 else 1e-6)
    sfa = a.aca_blocks(1e-5, 64, prec, g.FLAG_RECOMPRESS)
    sfb = b.aca_blocks(1e-5, 64, prec, g.FLAG_RECOMPRESS)
    assert sfa.rank_sum == sfb.rank_sum and sfa.aca_rank_sum == sfb.aca_rank_sum
    far = np.nonzero(a.get_tree()[1][:, 4])[0]
    for blk in far[::5]:
        for k in (0, 4, 8):
            Ua, Va = a.get_block_factors(int(blk), k)
            Ub, Vb = b.get_block_factors(int(blk), k)
            assert np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)


def _pca_tree(P, leaf, eta):
    """Cluster tree by principal-axis bisection of the centroids (the paper's
    split), block tree by eq. admissible on vertex boxes; in upload arrays."""
    begin, end, son = [], [], []
    perm = np.arange(P.n)

    def build(lo, hi):
        cid = len(begin)
        begin.append(lo); end.append(hi); son.append([-1, -1])
        if hi - lo <= leaf:
            return cid
        idx = perm[lo:hi]
        c = P.centroid[idx]
        w, v = np.linalg.eigh(np.cov((c - c.mean(0)).T))
        key = (c - c.mean(0)) @ v[:, -1]
        perm[lo:hi] = idx[np.lexsort((idx, key))]
        mid = lo + (hi - lo) // 2
        s0 = build(lo, mid)
        s1 = build(mid, hi)
        son[cid] = [s0, s1]
        return cid

    build(0, P.n)
    verts = np.stack([P.v0, P.v1, P.v2], 1)
    bmin = [verts[perm[b:e]].reshape(-1, 3).min(0) for b, e in zip(begin, end)]
    bmax = [verts[perm[b:e]].reshape(-1, 3).max(0) for b, e in zip(begin, end)]
    rows, cols, adm = [], [], []

    def rec(a, b):
        gap = np.maximum(0, np.maximum(bmin[a] - bmax[b], bmin[b] - bmax[a]))
        d = np.linalg.norm(gap)
        diam = min(np.linalg.norm(bmax[a] - bmin[a]), np.linalg.norm(bmax[b] - bmin[b]))
        ok = d > 0 and diam <= eta * d
        if ok or son[a][0] < 0 or son[b][0] < 0:
            rows.append(a); cols.append(b); adm.append(int(ok))
            return
        for x in son[a]:
            for y in son[b]:
                rec(x, y)

    rec(0, 0)
    return (perm.astype(np.int32), np.array(begin, np.int32), np.array(end, np.int32),
            np.array(son, np.int32), np.array(rows, np.int32), np.array(cols, np.int32),
            np.array(adm, np.uint8))


@pytest.mark.parametrize("prec,tol", [(g.C128, 1e-5), (g.C64, 1e-4)])
def test_pca_partition_product_matches_dense_oracle(prec, tol):
    xyz, tri = mesh.icosphere(3)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    P = Panels(xyz, tri)
    ctx = _ctx(xyz, tri, s)
    info = ctx.upload_cluster_tree(*_pca_tree(P, 20, 0.8))
    assert info.n_far > 0
    ctx.aca3d(1e-7, 1e-6, 40, prec)
    X = rhs.random_complex(len(s), P.n, 0)
    Xd = to_dev(X, prec).reshape(-1)
    Y = torch.zeros_like(Xd)
    ctx.compressed_matvec(g.PER_FREQUENCY, prec, Xd, Y)
    Yg = from_dev(Y).reshape(len(s), P.n)
    Yt = matvec.dense(entries.dense(P, s, 1.0), X)
    per_k = np.linalg.norm(Yg - Yt, axis=1) / np.linalg.norm(Yt, axis=1)
    assert per_k.max() <= tol, per_k.max()
