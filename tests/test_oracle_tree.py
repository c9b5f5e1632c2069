"""Pins of the oracle's cluster and block trees: the blocks partition the index
square exactly once, far blocks satisfy eq. admissible, near blocks do not (or
touch a leaf), the split rule and box geometry match brute force."""
import numpy as np
import pytest

from oracle.geometry import Panels
from oracle.tree import ClusterTree, admissible, block_tree
from synth import mesh


@pytest.mark.parametrize("gen,leaf,eta", [("sphere3", 64, 1.0), ("sphere3", 16, 0.8),
                                          ("housing", 32, 1.0), ("cube", 20, 0.8)])
def test_partition_and_admissibility(gen, leaf, eta):
    xyz, tri = {"sphere3": lambda: mesh.icosphere(3), "housing": lambda: mesh.fin_housing(1500),
                "cube": lambda: mesh.unit_cube(2)}[gen]()
    P = Panels(xyz, tri)
    T = ClusterTree(P, leaf)
    assert sorted(T.perm.tolist()) == list(range(P.n))
    # clusters: sons split the parent range, floor(n/2) first; leaves iff n <= leaf
    for c in range(len(T.begin)):
        n = T.end[c] - T.begin[c]
        if T.is_leaf(c):
            assert n <= leaf
        else:
            assert n > leaf
            s0, s1 = T.son0[c], T.son1[c]
            assert T.begin[s0] == T.begin[c] and T.end[s0] == T.begin[c] + n // 2
            assert T.begin[s1] == T.end[s0] and T.end[s1] == T.end[c]
        # box = all vertices of the cluster's triangles (brute force)
        idx = T.indices(c)
        pts = np.concatenate([P.v0[idx], P.v1[idx], P.v2[idx]])
        assert np.array_equal(T.bmin[c], pts.min(0)) and np.array_equal(T.bmax[c], pts.max(0))
    B = block_tree(T, eta)
    cover = np.zeros((P.n, P.n), dtype=np.int32)
    for a, b, adm in B:
        I, J = T.indices(a), T.indices(b)
        cover[np.ix_(I, J)] += 1
        if adm:
            assert min(T.diam(a), T.diam(b)) <= eta * T.dist(a, b) and T.dist(a, b) > 0
        else:
            assert not admissible(T, a, b, eta)
            assert T.is_leaf(a) or T.is_leaf(b)
    assert (cover == 1).all()


def test_split_axis_and_order():
    """The first split of an elongated point set is along its longest centroid
    extent, ordered by coordinate then index."""
    xyz, tri = mesh.fin_housing(1500)      # 0.3 m long in z, 0.24 m across
    P = Panels(xyz, tri)
    T = ClusterTree(P, 64)
    z = P.centroid[:, 2]
    first = T.perm[T.begin[T.son0[0]]:T.end[T.son0[0]]]
    second = T.perm[T.begin[T.son1[0]]:T.end[T.son1[0]]]
    assert z[first].max() <= z[second].min()
    order = np.lexsort((np.arange(P.n), z))
    assert np.array_equal(T.perm[:P.n // 2], order[:P.n // 2]) or \
        set(T.perm[:P.n // 2].tolist()) == set(order[:P.n // 2].tolist())


def test_box_distance_brute_force():
    xyz, tri = mesh.icosphere(3)
    P = Panels(xyz, tri)
    T = ClusterTree(P, 64)
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, b = rng.integers(0, len(T.begin), 2)
        # distance between boxes = min over box points: clamp one box's corners
        lo1, hi1, lo2, hi2 = T.bmin[a], T.bmax[a], T.bmin[b], T.bmax[b]
        gap = np.array([max(0.0, lo1[k] - hi2[k], lo2[k] - hi1[k]) for k in range(3)])
        assert abs(T.dist(a, b) - np.sqrt((gap ** 2).sum())) < 1e-15
        assert abs(T.diam(a) - np.linalg.norm(hi1 - lo1)) < 1e-15
