"""Synthetic inputs: meshes are closed and outward oriented, the cube meshes have
the node/element counts printed in Sec. 5.1, and the frequency sets have the
conjugate pairing the method relies on."""
import os

import numpy as np
import pytest

from synth import freq, mesh, rhs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cube_table():
    rows = []
    for line in open(os.path.join(GOLDEN, "cube_refinement.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(x) for x in line.split()])
    return rows


@pytest.mark.parametrize("level", [1, 2, 3])
def test_cube_counts_match_sec51_table(level):
    row = [r for r in _cube_table() if int(r[0]) == level][0]
    xyz, tri = mesh.unit_cube(level)
    assert len(xyz) == int(row[1]) and len(tri) == int(row[2])
    assert mesh.check_closed_oriented(xyz, tri)
    # dt / h = 0.6 in every row of the table
    assert abs(row[4] / row[3] - 0.6) < 1e-12


@pytest.mark.parametrize("sub", [0, 1, 2, 3])
def test_icosphere(sub):
    xyz, tri = mesh.icosphere(sub)
    assert len(tri) == 20 * 4 ** sub and len(xyz) == 10 * 4 ** sub + 2
    assert mesh.check_closed_oriented(xyz, tri)
    assert np.allclose(np.linalg.norm(xyz, axis=1), 1.0)


def test_fin_housing_closed():
    xyz, tri = mesh.fin_housing(3000)
    assert mesh.check_closed_oriented(xyz, tri)
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    assert area.min() > 0
    # enclosed volume: cylinder plus fins
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    expect = np.pi * 0.1 ** 2 * 0.3 + 24 * 0.01 * 0.02 * 0.3
    assert abs(vol - expect) / expect < 0.02


def test_frequency_sets():
    s = freq.bdf2_circle(32, 0.05, 1e-8 ** (1 / 32))
    assert s[0].imag == 0 and s[16].imag == 0
    assert abs(s[0].real - 10.6686) < 1e-4 and abs(s[16].real - 55.6559) < 1e-4
    for k in range(1, 32):
        assert s[32 - k] == np.conj(s[k])
    assert (s.real > 0).all()
    s = freq.steps_contour(128, 1e-4) / 343.0
    assert abs(s.real.min() - 4.17) < 0.01 and abs(s.real.max() - 105.16) < 0.01


def test_rhs_deterministic():
    a = rhs.random_complex(4, 10, 0)
    b = rhs.random_complex(4, 10, 0)
    assert np.array_equal(a, b) and a.dtype == np.complex128
    r = rhs.sample_rows(100, 20, 0)
    assert len(np.unique(r)) == 20
