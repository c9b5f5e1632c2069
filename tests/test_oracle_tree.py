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
    """dist(a, b) is the smallest distance between a point of box a and a point
    of box b (found here by bound-constrained minimisation from random starts,
    not by the gap formula), a lower bound of every vertex-to-vertex distance
    of the two clusters; diam(c) is the box diagonal, an upper bound of every
    vertex-to-vertex distance inside cluster c."""
    from scipy.optimize import minimize
    xyz, tri = mesh.icosphere(3)
    P = Panels(xyz, tri)
    T = ClusterTree(P, 64)
    rng = np.random.default_rng(0)

    def verts(c):
        idx = T.indices(c)
        return np.concatenate([P.v0[idx], P.v1[idx], P.v2[idx]])

    for _ in range(50):
        a, b = rng.integers(0, len(T.begin), 2)
        bounds = [(T.bmin[a][k], T.bmax[a][k]) for k in range(3)] + \
                 [(T.bmin[b][k], T.bmax[b][k]) for k in range(3)]
        best = np.inf
        for _ in range(4):
            z0 = np.array([rng.uniform(lo, hi) for lo, hi in bounds])
            r = minimize(lambda z: ((z[:3] - z[3:]) ** 2).sum(), z0,
                         jac=lambda z: np.concatenate([2 * (z[:3] - z[3:]), -2 * (z[:3] - z[3:])]),
                         bounds=bounds, method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-12})
            best = min(best, r.fun)
        assert abs(T.dist(a, b) - np.sqrt(max(best, 0.0))) <= 1e-6
        va, vb = verts(a), verts(b)
        dmin = np.sqrt(((va[:, None, :] - vb[None, :, :]) ** 2).sum(-1).min())
        assert T.dist(a, b) <= dmin + 1e-15
        dmax = np.sqrt(((va[:, None, :] - va[None, :, :]) ** 2).sum(-1).max())
        assert dmax <= T.diam(a) + 1e-15
        # the diagonal joins two corners of the box: it is attained by a pair of
        # box points, so it is the box's own diameter
        assert abs(T.diam(a) - np.linalg.norm(T.bmax[a] - T.bmin[a])) <= 1e-15
