"""GPU parity of the 3D-ACA (gcq_aca3d) and of the compressed products
(gcq_compressed_matvec, per-frequency and eq.-product modes) against the
oracle's 3D-ACA and compressed products on the same partition."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import aca3d, entries, matvec
from oracle.geometry import Panels
from synth import freq, mesh, rhs
from tests._gpu_common import from_dev, kpos_map, make_ctx, rel, to_dev
from tests._oracle_tree_blocks import oracle_tree

pytestmark = pytest.mark.gpu
TOLA, TOLF = 1e-6, 1e-5


def _problem():
    xyz, tri = mesh.icosphere(3)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    return xyz, tri, s


def _oracle_3d(P, T, B, s, K):
    return [aca3d.aca3d_mesh_block(P, T.indices(a), T.indices(b), s[K], 1.0, adm, TOLA, TOLF, 40)
            for a, b, adm in B]


@pytest.fixture(scope="module")
def setup():
    xyz, tri, s = _problem()
    P, T, B, perm, blocks = oracle_tree(xyz, tri, 32, 1.0)
    rep, conj, K, kpos = kpos_map(s)
    b3 = _oracle_3d(P, T, B, s, K)
    return xyz, tri, s, P, T, B, rep, conj, K, kpos, b3


@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_aca3d_blocks_match_oracle(setup, prec):
    xyz, tri, s, P, T, B, rep, conj, K, kpos, b3 = setup
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    st = ctx.aca3d(TOLA, TOLF, 40, prec)
    assert st.n_blocks == len(B)
    num = den = 0.0
    same = 0
    for b, Bo in enumerate(b3):
        freqs, fib, sl = ctx.get_aca3d_block(b, len(K))
        Tg = np.einsum("dk,dij->kij", fib, sl) if len(freqs) else 0.0
        To = Bo.tensor() if Bo.rank else 0.0
        num += np.linalg.norm(Tg - To) ** 2
        den += np.linalg.norm(To) ** 2
        same += len(freqs) == Bo.rank
        if prec == g.C128 and len(freqs) and Bo.rank:
            assert freqs[0] == 0
    err = np.sqrt(num / den)
    assert err <= (1e-5 if prec == g.C128 else 1e-4), err
    if prec == g.C128:
        assert same >= 0.9 * len(b3)


@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_compressed_products(setup, prec):
    xyz, tri, s, P, T, B, rep, conj, K, kpos, b3 = setup
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.aca3d(TOLA, TOLF, 40, prec)
    X = rhs.random_complex(len(s), P.n, 0)
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    Y = torch.zeros(len(s) * P.n, dtype=dt, device="cuda")
    Xd = to_dev(X, prec).reshape(-1)
    ctx.compressed_matvec(g.PER_FREQUENCY, prec, Xd, Y)
    Yg = from_dev(Y).reshape(len(s), P.n)
    Yo = matvec.compressed(b3, X, rep, conj, kpos)
    tol = 1e-5 if prec == g.C128 else 1e-4
    assert rel(Yg, Yo) <= tol, rel(Yg, Yo)
    # against the dense operator: the 3D-ACA's own approximation error
    Yt = matvec.dense(entries.dense(P, s, 1.0), X)
    assert rel(Yg, Yt) <= 1e-4
    # eq. product: the weighted sum equals the sum of the per-frequency columns
    y = torch.zeros(P.n, dtype=dt, device="cuda")
    ctx.compressed_matvec(g.WEIGHTED_SUM, prec, Xd, y)
    yg = from_dev(y)
    assert rel(yg, Yg.sum(0)) <= (1e-12 if prec == g.C128 else 1e-5)
    yo = matvec.weighted_sum(b3, X, rep, conj, kpos)
    assert rel(yg, yo) <= tol


def test_products_without_conjugate_symmetry(setup):
    xyz, tri, s, P, T, B, rep, conj, K, kpos, b3 = setup
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0, sym=False)
    ctx.aca3d(TOLA, TOLF, 40, g.C128)
    X = rhs.random_complex(len(s), P.n, 2)
    Y = torch.zeros(len(s) * P.n, dtype=torch.complex128, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C128, to_dev(X, g.C128).reshape(-1), Y)
    Yg = from_dev(Y).reshape(len(s), P.n)
    Yt = matvec.dense(entries.dense(P, s, 1.0), X)
    assert rel(Yg, Yt) <= 1e-4


@pytest.mark.parametrize("waves,stack", [((1, 1, 1, 1), 8), ((2, 2, 2, 2), 8), ((4, 4, 4, 4), 1),
                                         ((8, 8, 8, 8), 8), ((1, 2, 4, 8), 1)])
def test_aca3d_group_sizes(setup, waves, stack):
    """Every group size (waves per block) gives the oracle's 3D-ACA, also when
    the stacked slice factors start from a one-slice reservation and move."""
    xyz, tri, s, P, T, B, rep, conj, K, kpos, b3 = setup
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.set_tuning(aca3d_waves=waves, aca3d_stack_slices=stack)
    assert list(ctx.get_tuning().aca3d_waves) == list(waves)
    ctx.aca3d(TOLA, TOLF, 40, g.C128)
    num = den = 0.0
    same = 0
    nfar = 0
    for b, Bo in enumerate(b3):
        if not Bo.admissible:
            continue
        nfar += 1
        freqs, fib, sl = ctx.get_aca3d_block(b, len(K))
        Tg = np.einsum("dk,dij->kij", fib, sl) if len(freqs) else 0.0
        To = Bo.tensor() if Bo.rank else 0.0
        num += np.linalg.norm(Tg - To) ** 2
        den += np.linalg.norm(To) ** 2
        same += len(freqs) == Bo.rank
    assert nfar > 0
    err = np.sqrt(num / den)
    assert err <= 1e-5, err
    assert same >= 0.9 * nfar



@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_product_graph_replays_match_plain_launches(setup, prec):
    """The captured product graph, replayed several times with other work and
    synchronisations in between, gives the plain launches' result every time."""
    xyz, tri, s, P, T, B, rep, conj, K, kpos, b3 = setup
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.aca3d(TOLA, TOLF, 40, prec)
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    X = to_dev(rhs.random_complex(len(s), P.n, 0), prec).reshape(-1)
    X2 = to_dev(rhs.random_complex(len(s), P.n, 5), prec).reshape(-1)
    Y0 = torch.zeros(len(s) * P.n, dtype=dt, device="cuda")
    ctx.set_tuning(product_graph=0)
    ctx.compressed_matvec(g.PER_FREQUENCY, prec, X, Y0)
    ref = from_dev(Y0)
    ref2 = None
    tol = 1e-12 if prec == g.C128 else 1e-5
    Y = torch.empty_like(Y0)
    for rep_i in range(4):
        ctx.set_tuning(product_graph=1)
        Y.fill_(7.0)   # the same buffers every time: the same graph is replayed
        ctx.compressed_matvec(g.PER_FREQUENCY, prec, X, Y)
        assert rel(from_dev(Y), ref) <= tol, rep_i
        # eager work between the replays: a plain product on other buffers
        ctx.set_tuning(product_graph=0)
        Y2 = torch.zeros_like(Y0)
        ctx.compressed_matvec(g.PER_FREQUENCY, prec, X2, Y2)
        y2 = from_dev(Y2)
        if ref2 is None:
            ref2 = y2
        assert rel(y2, ref2) <= tol
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_aca3d_reuses_the_h_matrix_near_field(setup, prec):
    """After gcq_aca_blocks at the same frequencies and precision, the 3D-ACA
    reads the dense near-field entries the H-matrix holds instead of evaluating
    them again: every block's terms are those of a 3D-ACA run without it, and
    the far blocks still match the oracle."""
    xyz, tri, s, P, T, B, rep, conj, K, kpos, b3 = setup
    fresh = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    fresh.aca3d(TOLA, TOLF, 40, prec)
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.aca_blocks(TOLA, 64, prec, g.FLAG_RECOMPRESS)
    ctx.aca3d(TOLA, TOLF, 40, prec)
    assert ctx.kernel_ms("aca3d_tensor") == 0.0   # no entry evaluation of its own
    nnear = 0
    for b, Bo in enumerate(b3):
        f1, fib1, sl1 = fresh.get_aca3d_block(b, len(K))
        f2, fib2, sl2 = ctx.get_aca3d_block(b, len(K))
        assert list(f1) == list(f2), b
        np.testing.assert_array_equal(fib1, fib2)
        np.testing.assert_array_equal(sl1, sl2)
        nnear += not Bo.admissible
    assert nnear > 0
    # a change of precision makes it evaluate the entries again
    ctx.aca3d(TOLA, TOLF, 40, g.C64 if prec == g.C128 else g.C128)
    assert ctx.kernel_ms("aca3d_tensor") > 0.0
