"""Panel tables of a flat-triangle mesh (oracle; eq. geomapprox).

For each triangle tau_j: its vertices, area, centroid x_j (the collocation
point for the piecewise-constant basis psi_j), the longest edge h_j, the
far-field quadrature (7 points) and the near-field quadrature (7 points on each
of the 16 sub-triangles of two midpoint subdivisions).  Quadrature weights
include the area.
"""
from __future__ import annotations

import numpy as np

from . import quadrature


def sqnorm(d):
    """Squared Euclidean length of 3-vectors (last axis), summed x, y, z in order."""
    d = np.asarray(d, dtype=np.float64)
    return d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]


class Panels:
    def __init__(self, xyz, tri):
        xyz = np.asarray(xyz, dtype=np.float64)
        tri = np.asarray(tri, dtype=np.int64)
        self.n = len(tri)
        self.xyz = xyz
        self.tri = tri
        self.v0 = xyz[tri[:, 0]]
        self.v1 = xyz[tri[:, 1]]
        self.v2 = xyz[tri[:, 2]]
        cr = np.cross(self.v1 - self.v0, self.v2 - self.v0)
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.normal = cr / (2.0 * self.area[:, None])
        self.centroid = (self.v0 + self.v1 + self.v2) / 3.0
        e2 = np.stack([sqnorm(self.v1 - self.v0), sqnorm(self.v2 - self.v1),
                       sqnorm(self.v0 - self.v2)], axis=1)
        self.h2 = e2.max(axis=1)          # squared longest edge
        self.h = np.sqrt(self.h2)
        bary, w = quadrature.radon7()
        # far rule: (n, 7, 3) points and (n, 7) weights
        self.qp = (bary[None, :, 0:1] * self.v0[:, None, :]
                   + bary[None, :, 1:2] * self.v1[:, None, :]
                   + bary[None, :, 2:3] * self.v2[:, None, :])
        self.qw = w[None, :] * self.area[:, None]
        self._near = {}

    def near_rule(self, j: int):
        """112-point rule of panel j (two levels of midpoint subdivision)."""
        r = self._near.get(j)
        if r is None:
            r = quadrature.triangle_rule(self.v0[j], self.v1[j], self.v2[j], levels=2)
            self._near[j] = r
        return r
