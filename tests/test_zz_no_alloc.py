"""gcq_assemble_slices_noalloc (the entry point for callers that cannot
allocate device memory) against gcq_assemble_slices, through the C ABI: the
same entries bit for bit, on two calls in a row (the second smaller, so that
stale staging contents would show), in both precisions; requests beyond the
staging limit are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from synth import configs

pytestmark = pytest.mark.gpu


def _call(fn, ctx, rows, cols, fidx, prec, out):
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    return fn(ctx._h, vp(rows), len(rows), vp(cols), len(cols), vp(fidx), len(fidx), prec,
              C.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_noalloc_matches_assemble_slices(prec):
    cfg = configs.get("housing3k")
    ctx = g.Context(0)
    ctx.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
    ctx.set_frequencies(cfg["s"], True)
    ctx.build_cluster_tree(cfg["leaf"], cfg["eta"])
    n = len(cfg["tri"])
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    rng = np.random.default_rng(4)
    for nr, nc, nf in [(300, 700, 9), (37, 5, 2)]:   # the second call smaller than the first
        rows = rng.choice(n, nr, replace=False).astype(np.int32)
        cols = rng.choice(n, nc, replace=False).astype(np.int32)
        cols[0] = rows[0]                              # a self entry
        fidx = rng.choice(129, nf, replace=False).astype(np.int32)
        ref = torch.full((nf * nc * nr,), float("nan"), dtype=dt, device="cuda")
        out = torch.full_like(ref, float("nan"))
        assert _call(g.lib.gcq_assemble_slices, ctx, rows, cols, fidx, prec, ref) == 0
        assert _call(g.lib.gcq_assemble_slices_noalloc, ctx, rows, cols, fidx, prec, out) == 0
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b)
    # beyond the staging limit: refused on the host, nothing enqueued
    big = np.zeros(3_000_000, np.int32)
    one = np.zeros(1, np.int32)
    small = torch.zeros(1, dtype=dt, device="cuda")
    vp = lambda x: x.ctypes.data_as(C.c_void_p)
    rc = g.lib.gcq_assemble_slices_noalloc(ctx._h, vp(big), len(big), vp(one), 0, vp(one), 1, prec,
                                           C.c_void_p(small.data_ptr()))
    assert rc == 0   # an empty request (no columns) is a no-op
    rc = g.lib.gcq_assemble_slices_noalloc(ctx._h, vp(big), len(big), vp(one), 1, vp(one), 1, prec,
                                           C.c_void_p(small.data_ptr()))
    assert rc == -1   # GCQ_ERR_ARG: 12 MB of staging asked for
