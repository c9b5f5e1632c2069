"""Degenerate and edge cases of the GPU path against the oracle: a partition
without admissible blocks, odd and single frequency counts, zero inputs, the
frequency-rank cap, and ragged block sizes (leaf sizes that do not divide the
cluster sizes)."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import entries, matvec
from oracle.geometry import Panels
from synth import freq, mesh, rhs
from tests._gpu_common import from_dev, make_ctx, rel, to_dev

pytestmark = pytest.mark.gpu


def _dense_product(P, s, X, c=1.0):
    return matvec.dense(entries.dense(P, s, c), X)


def test_partition_without_admissible_blocks():
    xyz, tri = mesh.icosphere(1)              # 80 triangles, leaf 64: two touching halves
    s = freq.bdf2_circle(8, 0.05, 1e-8 ** (1 / 8))
    ctx = make_ctx(xyz, tri, 1.0, s, 64, 1.0)
    _, blocks = ctx.get_tree()
    assert int(blocks[:, 4].sum()) == 0
    st = ctx.aca_blocks(1e-5, 64, g.C128, g.FLAG_RECOMPRESS)
    assert st.n_pairs == 0
    st3 = ctx.aca3d(1e-6, 1e-6, 40, g.C128)
    assert st3.n_blocks == len(blocks)
    P = Panels(xyz, tri)
    X = rhs.random_complex(len(s), P.n, 0)
    Y = torch.zeros(len(s) * P.n, dtype=torch.complex128, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C128, to_dev(X, g.C128).reshape(-1), Y)
    assert rel(from_dev(Y).reshape(len(s), P.n), _dense_product(P, s, X)) <= 1e-5


@pytest.mark.parametrize("L", [1, 5])
def test_single_and_odd_frequency_counts(L):
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(L, 0.05, 1e-8 ** (1 / max(L, 2)))
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.aca3d(1e-6, 1e-6, 40, g.C128)
    P = Panels(xyz, tri)
    X = rhs.random_complex(L, P.n, 3)
    Y = torch.zeros(L * P.n, dtype=torch.complex128, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C128, to_dev(X, g.C128).reshape(-1), Y)
    assert rel(from_dev(Y).reshape(L, P.n), _dense_product(P, s, X)) <= 1e-4


def test_zero_inputs():
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(8, 0.05, 1e-8 ** (1 / 8))
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.aca3d(1e-5, 1e-5, 40, g.C64)
    n = len(tri)
    X = torch.zeros(8 * n, dtype=torch.complex64, device="cuda")
    Y = torch.full_like(X, 3.0)
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C64, X, Y)
    assert float(torch.abs(Y).max()) == 0.0
    B = torch.zeros(8 * n, dtype=torch.complex128, device="cuda")
    Xs = torch.full_like(B, 5.0)
    st = ctx.solve(B, Xs, rtol=1e-6, max_iter=20, restart=10, precision=g.C64)
    assert st.n_converged == st.n_systems == 8
    assert float(torch.abs(Xs).max()) == 0.0


def test_frequency_rank_cap_is_reported():
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    st = ctx.aca3d(1e-6, 1e-10, 1, g.C128)
    assert st.status == g.RANK_CAPPED
    assert st.rank_max == 1 and st.n_capped > 0


@pytest.mark.parametrize("leaf", [20, 48])
def test_ragged_block_sizes(leaf):
    """The finned housing at about 3000 triangles: cluster sizes that are not
    powers of two, blocks with ragged tiles; sampled rows against the oracle."""
    xyz, tri = mesh.fin_housing(3000)
    s = freq.steps_contour(4, 1e-4)
    c = 343.0
    ctx = make_ctx(xyz, tri, c, s, leaf, 1.0)
    _, blocks = ctx.get_tree()
    sizes = set((blocks[:, 1] - blocks[:, 0]).tolist())
    assert any(sz % 2 for sz in sizes)
    ctx.aca3d(1e-6, 1e-6, 40, g.C64)
    P = Panels(xyz, tri)
    L = len(s)
    X = rhs.random_complex(L, P.n, 1)
    Y = torch.zeros(L * P.n, dtype=torch.complex64, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C64, to_dev(X, g.C64).reshape(-1), Y)
    Yg = from_dev(Y).reshape(L, P.n)
    rows = rhs.sample_rows(P.n, 10, 2)
    A = entries.block(P, rows, np.arange(P.n), s, c)
    ref = np.einsum("kij,kj->ki", A, X)
    assert rel(Yg[:, rows], ref) <= 1e-4
