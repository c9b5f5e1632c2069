"""GPU parity of the double-layer entries (gcq_assemble_dlp_slices) against the
oracle (oracle.dlp): the whole 320-triangle sphere at all 32 frequencies,
ragged row/column subsets, and sampled rows and columns of the 41k-triangle
housing at 256 frequencies, in complex128 and complex64."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import dlp, entries
from oracle.geometry import Panels
from synth import configs, rhs

pytestmark = pytest.mark.gpu


def _ctx(cfg, leaf=64, eta=1.0):
    ctx = g.Context(0)
    ctx.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
    ctx.set_frequencies(cfg["s"], True)
    ctx.build_cluster_tree(leaf, eta)
    return ctx


def _assemble(ctx, rows, cols, fidx, prec):
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    out = torch.full((len(fidx) * len(cols) * len(rows),), np.nan, dtype=dt, device="cuda")
    ctx.assemble_dlp_slices(rows, cols, fidx, prec, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128).reshape(len(fidx), len(cols), len(rows)).transpose(0, 2, 1)


def _close(A, ref, rtol, atol_rel):
    """|A - ref| <= rtol |ref| + atol_rel max|ref| per frequency (entries of
    coplanar pairs vanish up to rounding)."""
    scale = np.abs(ref).reshape(len(ref), -1).max(axis=1)[:, None, None]
    return np.abs(A - ref) <= rtol * np.abs(ref) + atol_rel * scale


def test_sphere320_all_dlp_entries():
    cfg = configs.get("sphere320")
    P = Panels(cfg["xyz"], cfg["tri"])
    ref = dlp.dense(P, cfg["s"], cfg["c"])
    ctx = _ctx(cfg)
    idx = np.arange(320)
    fidx = np.arange(32)
    A = _assemble(ctx, idx, idx, fidx, g.C128)
    assert _close(A, ref, 1e-11, 1e-14).all()
    assert np.all(np.diagonal(A, axis1=1, axis2=2) == 0)
    A32 = _assemble(ctx, idx, idx, fidx, g.C64)
    err = np.linalg.norm((A32 - ref).reshape(32, -1), axis=1) / np.linalg.norm(ref.reshape(32, -1), axis=1)
    assert err.max() < 1e-5, err.max()
    near = np.array([[entries.tier(P, i, j) == entries.NEAR for j in range(320)] for i in range(320)])
    r32 = np.abs(A32 - ref) / np.abs(ref).max()
    assert r32[:, near].max() < 1e-7          # near tier in double on the complex64 path too


def test_dlp_ragged_subsets_and_empty():
    cfg = configs.get("sphere320")
    P = Panels(cfg["xyz"], cfg["tri"])
    ctx = _ctx(cfg)
    rng = np.random.default_rng(5)
    rows = rng.choice(320, 37, replace=False)
    cols = np.concatenate([rows[:5], rng.choice(320, 48, replace=False)])   # self pairs too
    fidx = np.array([0, 7, 16, 31])
    ref = dlp.block(P, rows, cols, cfg["s"][fidx], cfg["c"])
    A = _assemble(ctx, rows, cols, fidx, g.C128)
    assert _close(A, ref, 1e-11, 1e-14).all()
    out = torch.zeros(0, dtype=torch.complex128, device="cuda")
    ctx.assemble_dlp_slices(np.zeros(0, np.int32), cols, fidx, g.C128, out)   # empty: no work
    with pytest.raises(g.GcqError):                                         # column out of range
        ctx.assemble_dlp_slices([0, 1], [0, 400], [0], g.C128, torch.zeros(4, dtype=torch.complex128, device="cuda"))


def test_dlp_sphere_row_sums_follow_the_closed_form():
    """The library's row sums on the 320-triangle sphere against the closed form
    of the double layer of a constant density, at frequencies the mesh resolves
    (|s| R / c <= 3.6), to the discretisation error the oracle shows there."""
    cfg = configs.get("sphere320")
    s = np.array([1e-3, 0.5, 1.0, 2 + 1j, 3 - 2j])
    ctx = g.Context(0)
    ctx.upload_mesh(cfg["xyz"], cfg["tri"], 1.0)
    ctx.set_frequencies(s, False)
    ctx.build_cluster_tree(64, 1.0)
    idx = np.arange(320)
    A = _assemble(ctx, idx, idx, np.arange(len(s)), g.C128)
    err = np.abs(A.sum(-1) - dlp.sphere_constant(1.0, s, 1.0)[:, None]).max(axis=1)
    assert err[0] < 1e-5                       # Gauss's identity on the closed polyhedron
    assert np.all(err < [1e-5, 1e-3, 2e-3, 1e-2, 2e-2]), err


def test_housing_sampled_dlp_entries_full_size():
    cfg = configs.get("housing40k")
    P = Panels(cfg["xyz"], cfg["tri"])
    rows = rhs.sample_rows(P.n, 48, 0)
    cols = np.unique(np.concatenate([rows, rhs.sample_rows(P.n, 400, 1)]))
    fidx = np.array([0, 1, 64, 128, 200, 255])
    ref = dlp.block(P, rows, cols, cfg["s"][fidx], cfg["c"])
    ctx = _ctx(cfg)
    A = _assemble(ctx, rows, cols, fidx, g.C128)
    assert _close(A, ref, 1e-11, 1e-13).all()
    A32 = _assemble(ctx, rows, cols, fidx, g.C64)
    err = np.linalg.norm((A32 - ref).reshape(len(fidx), -1), axis=1) / np.linalg.norm(ref.reshape(len(fidx), -1), axis=1)
    assert err.max() < 1e-5, err


@pytest.fixture(scope="module")
def sphere1280():
    from synth import mesh
    xyz, tri = mesh.icosphere(3)
    P = Panels(xyz, tri)
    s = np.array([1.0, 2.0 + 1.0j, 5.0 - 3.0j])
    return xyz, tri, P, s, dlp.dense(P, s, 1.0)


@pytest.mark.parametrize("prec,tol,bound", [(g.C128, 1e-8, 1e-6), (g.C64, 1e-5, 1e-4)])
def test_dlp_h_matrix_product(sphere1280, prec, tol, bound):
    """Per-frequency ACA faces of the double layer (gcq_aca_blocks with
    GCQ_FLAG_DOUBLE_LAYER) applied by the H-matrix product against the
    oracle's dense double layer, on 1280 triangles at three frequencies."""
    xyz, tri, P, s, K = sphere1280
    ctx = g.Context(0)
    ctx.upload_mesh(xyz, tri, 1.0)
    ctx.set_frequencies(s, False)
    ctx.build_cluster_tree(32, 1.0)
    st = ctx.aca_blocks(tol, 64, prec, g.FLAG_RECOMPRESS | g.FLAG_DOUBLE_LAYER)
    assert st.n_pairs > 0 and st.n_capped == 0
    X = np.random.default_rng(8).standard_normal((len(s), P.n)) + 1j * np.random.default_rng(9).standard_normal((len(s), P.n))
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    Y = torch.zeros(len(s) * P.n, dtype=dt, device="cuda")
    ctx.compressed_matvec(g.PLAIN_H, prec, torch.from_numpy(X.reshape(-1)).to(dt).cuda(), Y)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().astype(np.complex128).reshape(len(s), P.n)
    ref = np.stack([K[k] @ X[k] for k in range(len(s))])
    err = np.linalg.norm(Yg - ref) / np.linalg.norm(ref)
    assert err <= bound, err
    with pytest.raises(g.GcqError):   # the rank model is the single layer's
        ctx.aca_blocks(tol, 64, prec, g.FLAG_DOUBLE_LAYER | g.FLAG_USE_PREDICTOR)


def test_single_layer_3d_aca_after_double_layer_faces(sphere1280):
    """A 3D-ACA after double-layer faces rebuilds its near field with the single
    layer (the faces' near blocks are not reused)."""
    xyz, tri, P, s, _ = sphere1280
    ctx = g.Context(0)
    ctx.upload_mesh(xyz, tri, 1.0)
    ctx.set_frequencies(s, False)
    ctx.build_cluster_tree(32, 1.0)
    ctx.aca_blocks(1e-8, 64, g.C128, g.FLAG_RECOMPRESS | g.FLAG_DOUBLE_LAYER)
    ctx.aca3d(1e-8, 1e-8, 64, g.C128)
    X = np.random.default_rng(10).standard_normal((len(s), P.n)).astype(np.complex128)
    Y = torch.zeros(len(s) * P.n, dtype=torch.complex128, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C128, torch.from_numpy(X.reshape(-1)).cuda(), Y)
    torch.cuda.synchronize()
    V = entries.dense(P, s, 1.0)
    ref = np.stack([V[k] @ X[k] for k in range(len(s))])
    Yg = Y.cpu().numpy().reshape(len(s), P.n)
    assert np.linalg.norm(Yg - ref) / np.linalg.norm(ref) <= 1e-6


@pytest.mark.parametrize("prec,tol,bound", [(g.C128, 1e-8, 1e-6), (g.C64, 1e-5, 1e-4)])
def test_dlp_3d_aca_product(sphere1280, prec, tol, bound):
    """3D-ACA of the double layer (gcq_aca3d with GCQ_FLAG_DOUBLE_LAYER) and the
    per-frequency product against the oracle's dense double layer; after it, a
    single-layer 3D-ACA on the same context is the single layer again."""
    xyz, tri, P, s, K = sphere1280
    ctx = g.Context(0)
    ctx.upload_mesh(xyz, tri, 1.0)
    ctx.set_frequencies(s, False)
    ctx.build_cluster_tree(32, 1.0)
    st = ctx.aca3d(tol, tol, 64, prec, g.FLAG_DOUBLE_LAYER)
    assert st.n_blocks > 0 and st.n_capped == 0
    rng = np.random.default_rng(12)
    X = rng.standard_normal((len(s), P.n)) + 1j * rng.standard_normal((len(s), P.n))
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    Xd = torch.from_numpy(X.reshape(-1)).to(dt).cuda()
    Y = torch.zeros(len(s) * P.n, dtype=dt, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, prec, Xd, Y)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().astype(np.complex128).reshape(len(s), P.n)
    ref = np.stack([K[k] @ X[k] for k in range(len(s))])
    err = np.linalg.norm(Yg - ref) / np.linalg.norm(ref)
    assert err <= bound, err
    if prec == g.C128:
        ctx.aca3d(tol, tol, 64, prec)
        ctx.compressed_matvec(g.PER_FREQUENCY, prec, Xd, Y)
        torch.cuda.synchronize()
        V = entries.dense(P, s, 1.0)
        refv = np.stack([V[k] @ X[k] for k in range(len(s))])
        Yv = Y.cpu().numpy().reshape(len(s), P.n)
        assert np.linalg.norm(Yv - refv) / np.linalg.norm(refv) <= bound


def test_dlp_3d_aca_with_conjugate_symmetry():
    """The double layer's 3D-ACA over the 32-point BDF2 set with conjugate
    symmetry (K(conj s) = conj K(s): only 17 frequencies approximated), every
    frequency's product against the oracle's dense double layer."""
    cfg = configs.get("sphere320")
    P = Panels(cfg["xyz"], cfg["tri"])
    K = dlp.dense(P, cfg["s"], cfg["c"])
    ctx = _ctx(cfg, leaf=16)
    st = ctx.aca3d(1e-8, 1e-8, 64, g.C128, g.FLAG_DOUBLE_LAYER)
    assert st.n_blocks > 0
    L = len(cfg["s"])
    rng = np.random.default_rng(14)
    X = rng.standard_normal((L, P.n)) + 1j * rng.standard_normal((L, P.n))
    Y = torch.zeros(L * P.n, dtype=torch.complex128, device="cuda")
    ctx.compressed_matvec(g.PER_FREQUENCY, g.C128, torch.from_numpy(X.reshape(-1)).cuda(), Y)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().reshape(L, P.n)
    ref = np.stack([K[k] @ X[k] for k in range(L)])
    err = np.linalg.norm(Yg - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-6, err.max()
