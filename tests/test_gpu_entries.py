"""GPU parity of the entry evaluation (gcq_assemble_slices) against the oracle:
the whole 320-triangle sphere at all 32 frequencies, and sampled rows and
columns of the 41k-triangle housing at 256 frequencies, in complex128 and
complex64."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import entries
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
    out = torch.zeros(len(fidx) * len(cols) * len(rows), dtype=dt, device="cuda")
    ctx.assemble_slices(rows, cols, fidx, prec, out)
    torch.cuda.synchronize()
    # (f, col, row) -> (f, row, col)
    return out.cpu().numpy().astype(np.complex128).reshape(len(fidx), len(cols), len(rows)).transpose(0, 2, 1)


def test_sphere320_all_entries():
    cfg = configs.get("sphere320")
    P = Panels(cfg["xyz"], cfg["tri"])
    ref = entries.dense(P, cfg["s"], cfg["c"])
    ctx = _ctx(cfg)
    idx = np.arange(320)
    fidx = np.arange(32)
    A = _assemble(ctx, idx, idx, fidx, g.C128)
    rel = np.abs(A - ref) / np.abs(ref)
    assert rel.max() < 1e-11, rel.max()
    A32 = _assemble(ctx, idx, idx, fidx, g.C64)
    err = np.linalg.norm((A32 - ref).reshape(32, -1), axis=1) / np.linalg.norm(ref.reshape(32, -1), axis=1)
    assert err.max() < 1e-5, err.max()
    # self and near entries are computed in double even on the complex64 path
    near = np.array([[entries.tier(P, i, j) != entries.FAR for j in range(320)] for i in range(320)])
    r32 = np.abs(A32 - ref) / np.abs(ref)
    assert r32[:, near].max() < 1e-6


def test_housing_sampled_entries_full_size():
    cfg = configs.get("housing40k")
    P = Panels(cfg["xyz"], cfg["tri"])
    rows = rhs.sample_rows(P.n, 48, 0)
    cols = np.unique(np.concatenate([rows, rhs.sample_rows(P.n, 400, 1)]))   # self + far + some near
    fidx = np.array([0, 1, 64, 128, 200, 255])
    ref = entries.block(P, rows, cols, cfg["s"][fidx], cfg["c"])
    ctx = _ctx(cfg)
    A = _assemble(ctx, rows, cols, fidx, g.C128)
    assert (np.abs(A - ref) <= 1e-11 * np.abs(ref) + 1e-300).all()
    A32 = _assemble(ctx, rows, cols, fidx, g.C64)
    err = np.linalg.norm((A32 - ref).reshape(len(fidx), -1), axis=1) / np.linalg.norm(ref.reshape(len(fidx), -1), axis=1)
    assert err.max() < 1e-5, err


def test_assemble_errors_and_empty():
    cfg = configs.get("sphere320")
    ctx = _ctx(cfg)
    out = torch.zeros(4, dtype=torch.complex128, device="cuda")
    with pytest.raises(g.GcqError):
        ctx.assemble_slices([0, 1], [0, 400], [0], g.C128, out)     # column out of range
    with pytest.raises(g.GcqError):
        ctx.assemble_slices([0, 1], [0, 1], [40], g.C128, out)      # frequency out of range
    host = np.zeros(4, np.complex128)
    rc = g.lib.gcq_assemble_slices(ctx._h, np.array([0, 1], np.int32).ctypes.data, 2,
                                   np.array([0, 1], np.int32).ctypes.data, 2,
                                   np.array([0], np.int32).ctypes.data, 1, 0, host.ctypes.data)
    assert rc == -1                                                   # host pointer rejected
    # empty request is a no-op
    ctx.assemble_slices(np.zeros(0, np.int32), [0], [0], g.C128, torch.zeros(0, dtype=torch.complex128, device="cuda"))
