"""Seeded, deterministic surface-mesh generators (input data only).

These meshes stand in for the paper's workloads (the unit sphere used for the
closed-form check, and a finned machine housing shaped like the electric-machine
example of Sec. 5.2, whose geometry is not published).  They hold none of the
boundary-element arithmetic: they only produce vertex coordinates and triangle
connectivity of a closed, outward-oriented surface made of flat triangles
(eq. geomapprox).

Every function returns ``(xyz, tri)`` with ``xyz`` float64 ``(nv, 3)`` and
``tri`` int32 ``(nt, 3)``.
"""
from __future__ import annotations

import math

import numpy as np


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
         [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
         [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def icosphere(subdiv: int, radius: float = 1.0):
    """Icosahedron refined ``subdiv`` times by 4-fold midpoint splitting, vertices
    projected onto the sphere of the given radius.  20*4**subdiv triangles,
    10*4**subdiv + 2 vertices, outward orientation."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = (np.asarray(verts[a]) + np.asarray(verts[b])) * 0.5
                m /= np.linalg.norm(m)
                verts.append(tuple(m))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
    xyz = np.asarray(verts, dtype=np.float64) * radius
    tri = f.astype(np.int32)
    # orient outward (the icosahedron table above is consistently oriented;
    # enforce it explicitly so that the generator is self-checking)
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, (a + b + c)) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return xyz, tri


def _ring_zip(outer, inner):
    """Triangulate the annulus between two closed vertex rings whose vertices are
    ordered by increasing polar angle (both start near angle 0).  ``outer`` and
    ``inner`` are lists of global vertex ids with an ``angle`` lookup supplied as
    tuples (id, angle).  Triangles are returned counter-clockwise in the plane."""
    tris = []
    no, ni = len(outer), len(inner)
    io = ii = 0
    while io < no or ii < ni:
        o0, ao0 = outer[io % no]
        i0, ai0 = inner[ii % ni]
        o1, ao1 = outer[(io + 1) % no]
        i1, ai1 = inner[(ii + 1) % ni]
        ao1 += 2 * math.pi if io + 1 >= no else 0.0
        ai1 += 2 * math.pi if ii + 1 >= ni else 0.0
        if ii >= ni or (io < no and ao1 <= ai1):
            tris.append((o0, o1, i0))  # outer edge advances
            io += 1
        else:
            tris.append((o0, i1, i0))  # inner edge advances
            ii += 1
    return tris


def fin_housing(target_n: int = 40960, radius: float = 0.1, length: float = 0.3,
                n_fins: int = 24, fin_thick: float = 0.01, fin_height: float = 0.02):
    """Closed finned cylinder: radius ``radius``, axial length ``length``, with
    ``n_fins`` equally spaced axial rectangular fins of tangential thickness
    ``fin_thick`` and radial height ``fin_height`` over the full length.  The
    cross-section outline is extruded along z; each end cap is a disk meshed by
    concentric vertex rings (count proportional to radius, central fan) plus a
    small structured grid per fin.  The mesh size is chosen so that the triangle
    count is close to ``target_n``; the exact count is whatever results."""
    R = radius
    half = fin_thick / 2.0
    alpha = math.asin(half / R)                       # angular half-width of a fin base
    perim = 2 * math.pi * R + n_fins * (2 * fin_height)
    area = perim * length + 2 * (math.pi * R * R + n_fins * fin_thick * fin_height)
    h = math.sqrt(2.0 * area / target_n)              # structured-grid triangles: area ~ h^2/2

    n_side = max(1, round(fin_height / h))            # segments up a fin side
    n_top = max(1, round(fin_thick / h))              # segments across a fin top
    gap = 2 * math.pi / n_fins - 2 * alpha            # arc between two fins
    n_arc = max(1, round(gap * R / h))
    n_z = max(1, round(length / h))

    # ---- 2D outline (counter-clockwise), with a marker of which points lie on the circle
    pts2, on_circle = [], []
    for f in range(n_fins):
        th = 2 * math.pi * f / n_fins
        ct, st = math.cos(th), math.sin(th)
        er, et = np.array([ct, st]), np.array([-st, ct])  # radial / tangential unit vectors
        base = math.sqrt(R * R - half * half)
        top = R + fin_height
        # right side of the fin (tangential -half) going up, top going left, left side going down
        for k in range(n_side):
            rr = base + (top - base) * k / n_side
            pts2.append(er * rr - et * half); on_circle.append(k == 0)
        for k in range(n_top):
            tt = -half + fin_thick * k / n_top
            pts2.append(er * top + et * tt); on_circle.append(False)
        for k in range(n_side):
            rr = top - (top - base) * k / n_side
            pts2.append(er * rr + et * half); on_circle.append(False)
        # the left base point begins the arc to the next fin
        a0 = th + alpha
        for k in range(n_arc):
            a = a0 + gap * k / n_arc
            pts2.append(np.array([R * math.cos(a), R * math.sin(a)])); on_circle.append(True)
    pts2 = np.asarray(pts2)
    m = len(pts2)

    verts = []
    tris = []
    # ---- side wall: rings at z_k
    for k in range(n_z + 1):
        z = length * k / n_z
        for p in pts2:
            verts.append((p[0], p[1], z))
    for k in range(n_z):
        for i in range(m):
            a = k * m + i
            b = k * m + (i + 1) % m
            c = (k + 1) * m + (i + 1) % m
            d = (k + 1) * m + i
            # outward normal for a CCW outline extruded in +z: (a, b, c), (a, c, d)
            tris += [(a, b, c), (a, c, d)]

    # ---- caps
    def cap(z_level, ring_ids, flip):
        # ring_ids: ids of the outline vertices at this z (index i -> ring_ids[i])
        loc = []
        circle_ids = [(ring_ids[i], math.atan2(pts2[i][1], pts2[i][0]) % (2 * math.pi))
                      for i in range(m) if on_circle[i]]
        circle_ids.sort(key=lambda t: t[1])
        # fins: structured (n_side x n_top) grid spanning each fin rectangle in the cap plane
        idx_of = {}
        for f in range(n_fins):
            off = f * (2 * n_side + n_top + n_arc)
            right = [off + k for k in range(n_side)] + [off + n_side]        # right side incl. top corner
            left = [off + n_side + n_top + n_side - k for k in range(n_side + 1)]  # left side bottom..top
            left[0] = (off + 2 * n_side + n_top) % m                           # left base = first arc point
            left[-1] = off + n_side + n_top                                    # top-left corner
            # grid rows j = 0..n_side (base..top), columns t = 0..n_top (right..left)
            grid = [[None] * (n_top + 1) for _ in range(n_side + 1)]
            for j in range(n_side + 1):
                grid[j][0] = ring_ids[right[j]]
                grid[j][n_top] = ring_ids[left[j]]
            for t in range(n_top + 1):
                grid[n_side][t] = ring_ids[(off + n_side + t) % m] if t < n_top else ring_ids[left[-1]]
            for j in range(n_side):
                for t in range(1, n_top):
                    pr = np.asarray(verts[grid[j][0]][:2])
                    pl = np.asarray(verts[grid[j][n_top]][:2])
                    q = pr + (pl - pr) * t / n_top
                    verts.append((q[0], q[1], z_level))
                    grid[j][t] = len(verts) - 1
            for j in range(n_side):
                for t in range(n_top):
                    a, b = grid[j][t], grid[j][t + 1]
                    c, d = grid[j + 1][t + 1], grid[j + 1][t]
                    loc += [(a, d, c), (a, c, b)]
            idx_of[f] = [grid[0][t] for t in range(n_top + 1)]
            # the fin base (right->left) is now an outer-ring polyline on the disk
        # disk outer ring: circle points plus the interior fin-base points, by angle
        ring = list(circle_ids)
        for f in range(n_fins):
            for t in range(1, n_top):
                vid = idx_of[f][t]
                x, y = verts[vid][0], verts[vid][1]
                ring.append((vid, math.atan2(y, x) % (2 * math.pi)))
        ring.sort(key=lambda t: t[1])
        # concentric inner rings, vertex count proportional to radius
        n_out = len(ring)
        n_rings = max(1, round(R / h))
        prev = ring
        for k in range(n_rings - 1, 0, -1):
            rr = R * k / n_rings
            nk = max(6, round(n_out * k / n_rings))
            cur = []
            for q in range(nk):
                a = 2 * math.pi * (q + 0.5 * (k % 2)) / nk
                verts.append((rr * math.cos(a), rr * math.sin(a), z_level))
                cur.append((len(verts) - 1, a % (2 * math.pi)))
            cur.sort(key=lambda t: t[1])
            loc += _ring_zip(prev, cur)
            prev = cur
        verts.append((0.0, 0.0, z_level))
        cid = len(verts) - 1
        for q in range(len(prev)):
            a, b = prev[q][0], prev[(q + 1) % len(prev)][0]
            loc.append((a, b, cid))
        # loc triangles are CCW seen from +z; the top cap keeps them, the bottom flips
        for t in loc:
            tris.append((t[0], t[2], t[1]) if flip else t)

    cap(0.0, list(range(m)), flip=True)
    cap(length, [n_z * m + i for i in range(m)], flip=False)

    xyz = np.asarray(verts, dtype=np.float64)
    tri = np.asarray(tris, dtype=np.int64)
    # drop unused vertices and renumber
    used = np.zeros(len(xyz), bool)
    used[tri.ravel()] = True
    remap = -np.ones(len(xyz), np.int64)
    remap[used] = np.arange(used.sum())
    return xyz[used], remap[tri].astype(np.int32)


def unit_cube(level: int):
    """Unit cube [-0.5, 0.5]^3 centred at the origin (Sec. 5.1) with
    96*4**(level-1) triangles: each face is a grid of 2**level x 2**level squares
    of side h = 2**-level, each square cut into four triangles through its
    centre.  This reproduces the element and node counts of the refinement table
    of Sec. 5.1 (nodes = elements/2 + 2 for a closed triangulation)."""
    n = 2 ** level
    verts = {}
    tris = []

    def vid(p):
        key = tuple(int(round(c * 4 * n)) for c in p)
        if key not in verts:
            verts[key] = len(verts)
        return verts[key]

    for axis in range(3):
        for sgn in (-1.0, 1.0):
            u, w = [a for a in range(3) if a != axis]

            def P(a, b):
                p = [0.0, 0.0, 0.0]
                p[axis] = 0.5 * sgn
                p[u] = -0.5 + a / n
                p[w] = -0.5 + b / n
                return vid(p)

            for i in range(n):
                for j in range(n):
                    a, b, c, d = P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)
                    m = P(i + 0.5, j + 0.5)
                    tris += [(a, b, m), (b, c, m), (c, d, m), (d, a, m)]
    xyz = np.zeros((len(verts), 3))
    for key, k in verts.items():
        xyz[k] = np.asarray(key, dtype=np.float64) / (4 * n)
    tri = np.asarray(tris, dtype=np.int32)
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(b - a, c - a)
    ctr = (a + b + c) / 3.0
    flip = np.einsum("ij,ij->i", nrm, ctr) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return xyz, tri


def check_closed_oriented(xyz, tri):
    """True if every directed edge appears exactly once and its reverse exactly
    once (closed, consistently oriented 2-manifold) and the enclosed volume is
    positive (outward normals)."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    fwd = set(map(tuple, e.tolist()))
    if len(fwd) != len(e):
        return False
    for a, b in fwd:
        if (b, a) not in fwd:
            return False
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    return vol > 0
