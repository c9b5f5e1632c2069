"""Cluster tree and block cluster tree (oracle; Sec. 4, eq. admissible).

The paper bisects index sets by principal component analysis with a minimal
leaf size b_min and classifies blocks by min(diam) <= eta dist.  It defines
neither diam/dist nor the recursion; the reading used here (and by the
library):

  split   axis = longest extent of the bounding box of the cluster's centroids
          (ties x < y < z); order the cluster by (centroid coordinate on that
          axis, original index); the first son takes floor(n/2) indices.
          A cluster with n <= leaf_size is a leaf.
  boxes   axis-aligned box of all vertices of the cluster's triangles;
          diam = box diagonal; dist = Euclidean distance between the boxes.
  blocks  starting from (root, root), depth first: admissible (dist > 0 and
          min(diam) <= eta dist, evaluated on squares:
          min(diam^2) <= (eta*eta) dist^2) -> far leaf; otherwise, if either cluster is a
          leaf -> near leaf; otherwise recurse into the 2 x 2 son pairs in the
          order (s0,t0), (s0,t1), (s1,t0), (s1,t1).
"""
from __future__ import annotations

import numpy as np

from .geometry import sqnorm


class ClusterTree:
    def __init__(self, P, leaf_size: int):
        self.leaf_size = leaf_size
        self.perm = np.arange(P.n, dtype=np.int64)
        self.begin, self.end, self.son0, self.son1 = [], [], [], []
        self.bmin, self.bmax = [], []
        cen = P.centroid
        # vertices of each triangle (n, 3, 3)
        tv = np.stack([P.v0, P.v1, P.v2], axis=1)

        def build(lo: int, hi: int) -> int:
            cid = len(self.begin)
            self.begin.append(lo); self.end.append(hi)
            self.son0.append(-1); self.son1.append(-1)
            idx = self.perm[lo:hi]
            pts = tv[idx].reshape(-1, 3)
            self.bmin.append(pts.min(axis=0)); self.bmax.append(pts.max(axis=0))
            n = hi - lo
            if n <= leaf_size:
                return cid
            c = cen[idx]
            ext = c.max(axis=0) - c.min(axis=0)
            axis = int(np.argmax(ext))          # first maximum: x < y < z on ties
            order = np.lexsort((idx, c[:, axis]))  # primary key coordinate, then index
            self.perm[lo:hi] = idx[order]
            mid = lo + n // 2
            s0 = build(lo, mid)
            s1 = build(mid, hi)
            self.son0[cid] = s0
            self.son1[cid] = s1
            return cid

        build(0, P.n)
        self.begin = np.array(self.begin, np.int64)
        self.end = np.array(self.end, np.int64)
        self.son0 = np.array(self.son0, np.int64)
        self.son1 = np.array(self.son1, np.int64)
        self.bmin = np.array(self.bmin)
        self.bmax = np.array(self.bmax)

    def is_leaf(self, c: int) -> bool:
        return self.son0[c] < 0

    def indices(self, c: int):
        return self.perm[self.begin[c]:self.end[c]]

    def diam2(self, c: int) -> float:
        return float(sqnorm(self.bmax[c] - self.bmin[c]))

    def dist2(self, a: int, b: int) -> float:
        gap = np.maximum(0.0, np.maximum(self.bmin[a] - self.bmax[b], self.bmin[b] - self.bmax[a]))
        return float(sqnorm(gap))

    def diam(self, c: int) -> float:
        return float(np.sqrt(self.diam2(c)))

    def dist(self, a: int, b: int) -> float:
        return float(np.sqrt(self.dist2(a, b)))


def admissible(T: ClusterTree, a: int, b: int, eta: float) -> bool:
    d2 = T.dist2(a, b)
    return d2 > 0.0 and min(T.diam2(a), T.diam2(b)) <= (eta * eta) * d2


def block_tree(T: ClusterTree, eta: float):
    """List of (row_cluster, col_cluster, admissible) leaves in depth-first order."""
    out = []

    def rec(a: int, b: int):
        if admissible(T, a, b, eta):
            out.append((a, b, True))
        elif T.is_leaf(a) or T.is_leaf(b):
            out.append((a, b, False))
        else:
            for sa in (T.son0[a], T.son1[a]):
                for sb in (T.son0[b], T.son1[b]):
                    rec(int(sa), int(sb))

    rec(0, 0)
    return out
