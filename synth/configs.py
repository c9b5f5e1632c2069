"""The synthetic workloads, by name.  Each returns a dict with the mesh, the
frequency set and the run parameters; nothing here evaluates the method.

  sphere320      icosphere subdivision 2 (320 triangles), R = 1, c = 1,
                 L = 32 BDF2 points, dt = 0.05, lam = 1e-8**(1/32)
  sphere20480    icosphere subdivision 5 (20480 triangles), c = 1, leaf 64,
                 eta = 1, ACA tol 1e-5, L = 64 points (N = 32, dt = 0.02)
  housing40k     finned housing (R = 0.1 m, length 0.3 m, 24 fins 0.01 x 0.02 m),
                 about 40k triangles, c = 343 m/s, L = 256 (N = 128, dt = 1e-4 s)
  housing80k     the same housing at about 80k triangles
"""
from __future__ import annotations

from . import mesh, freq


def get(name: str) -> dict:
    if name == "sphere320":
        xyz, tri = mesh.icosphere(2, 1.0)
        s = freq.bdf2_circle(32, 0.05, 1e-8 ** (1.0 / 32))
        return dict(name=name, xyz=xyz, tri=tri, s=s, c=1.0, leaf=64, eta=1.0, tol=1e-5)
    if name == "sphere20480":
        xyz, tri = mesh.icosphere(5, 1.0)
        s = freq.steps_contour(32, 0.02)
        return dict(name=name, xyz=xyz, tri=tri, s=s, c=1.0, leaf=64, eta=1.0, tol=1e-5)
    if name.startswith("sphere"):
        sub = {"sphere1280": 3, "sphere5120": 4}[name]
        xyz, tri = mesh.icosphere(sub, 1.0)
        s = freq.steps_contour(32, 0.02)
        return dict(name=name, xyz=xyz, tri=tri, s=s, c=1.0, leaf=64, eta=1.0, tol=1e-5)
    if name == "housing40k":
        xyz, tri = mesh.fin_housing(40960)
        s = freq.steps_contour(128, 1e-4)
        return dict(name=name, xyz=xyz, tri=tri, s=s, c=343.0, leaf=64, eta=1.0, tol=1e-5)
    if name == "housing80k":
        xyz, tri = mesh.fin_housing(81920)
        s = freq.steps_contour(128, 1e-4)
        return dict(name=name, xyz=xyz, tri=tri, s=s, c=343.0, leaf=64, eta=1.0, tol=1e-5)
    if name == "housing3k":
        xyz, tri = mesh.fin_housing(3000)
        s = freq.steps_contour(128, 1e-4)
        return dict(name=name, xyz=xyz, tri=tri, s=s, c=343.0, leaf=64, eta=1.0, tol=1e-5)
    raise KeyError(name)
