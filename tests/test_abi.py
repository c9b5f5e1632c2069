"""The C ABI without a GPU: the library loads and exports every entry point
include/gcqbem.h declares; a host-only context builds exactly the oracle's
cluster and block trees; argument and call-order errors are reported."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2505_00715_amd as g
from synth import configs, freq, mesh
from tests._oracle_tree_blocks import oracle_tree

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "gcqbem.h")


def test_exports_every_declared_symbol():
    decl = set(re.findall(r"GCQ_API\s+[\w\s\*]+?\b(gcq_\w+)\s*\(", open(HEADER).read()))
    assert len(decl) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (gcq_\w+)", out))
    assert decl <= exported, decl - exported
    for name in decl:
        getattr(g.lib, name)


@pytest.mark.parametrize("name,leaf,eta", [("sphere320", 64, 1.0), ("sphere320", 16, 0.8),
                                           ("sphere5120", 64, 1.0), ("housing3k", 32, 1.0),
                                           ("housing3k", 20, 0.8)])
def test_host_tree_matches_oracle_exactly(name, leaf, eta):
    cfg = configs.get(name)
    ctx = g.Context(-1)
    ctx.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
    info = ctx.build_cluster_tree(leaf, eta)
    perm, blocks = ctx.get_tree()
    _, T, B, operm, oblocks = oracle_tree(cfg["xyz"], cfg["tri"], leaf, eta)
    assert np.array_equal(perm, operm)
    assert np.array_equal(blocks, oblocks)
    assert info.n_blocks == len(B) and info.n_far == int(oblocks[:, 4].sum())
    assert info.n_clusters == len(T.begin)
    ctx.destroy()


def test_cube_tree_matches_oracle():
    xyz, tri = mesh.unit_cube(3)
    ctx = g.Context(-1)
    ctx.upload_mesh(xyz, tri, 1.0)
    ctx.build_cluster_tree(20, 0.8)
    perm, blocks = ctx.get_tree()
    _, _, _, operm, oblocks = oracle_tree(xyz, tri, 20, 0.8)
    assert np.array_equal(perm, operm) and np.array_equal(blocks, oblocks)


def test_argument_and_state_errors():
    ctx = g.Context(-1)
    xyz, tri = mesh.icosphere(1)
    with pytest.raises(g.GcqError) as e:
        ctx.build_cluster_tree(16, 1.0)
    assert e.value.code == -4                       # GCQ_ERR_STATE: no mesh yet
    bad = tri.copy(); bad[0, 0] = len(xyz)
    with pytest.raises(g.GcqError) as e:
        ctx.upload_mesh(xyz, bad, 1.0)
    assert e.value.code == -1
    with pytest.raises(g.GcqError) as e:
        ctx.upload_mesh(xyz, tri, -1.0)
    assert e.value.code == -1
    deg = tri.copy(); deg[0, 2] = deg[0, 1]         # zero-area triangle
    with pytest.raises(g.GcqError) as e:
        ctx.upload_mesh(xyz, deg, 1.0)
    assert e.value.code == -5
    ctx.upload_mesh(xyz, tri, 1.0)
    with pytest.raises(g.GcqError) as e:
        ctx.set_frequencies(np.array([1.0 + 1j, -0.5 + 0j]))
    assert e.value.code == -1                       # Re s <= 0
    ctx.set_frequencies(freq.bdf2_circle(8, 0.05, 0.5))
    with pytest.raises(g.GcqError) as e:
        ctx.build_cluster_tree(0, 1.0)
    assert e.value.code == -1
    ctx.build_cluster_tree(16, 1.0)
    # device work on a host-only context is a state error
    rc = g.lib.gcq_aca3d(ctx._h, 1e-5, 1e-5, 10, 0, 0, None)
    assert rc < 0
    with pytest.raises(g.GcqError) as e:            # no 3D-ACA yet
        ctx.aca3d_ranks()
    assert e.value.code == -4
    assert g.lib.gcq_destroy(None) == 0
    ctx.destroy()


def test_tuning_roundtrip_and_rejection():
    ctx = g.Context(-1)
    assert list(ctx.get_tuning().aca3d_waves) == [4, 4, 4, 4]
    assert ctx.get_tuning().aca3d_stack_slices == 8
    ctx.set_tuning(aca3d_waves=(1, 1, 2, 4), aca3d_stack_slices=2)
    assert list(ctx.get_tuning().aca3d_waves) == [1, 1, 2, 4]
    with pytest.raises(g.GcqError):
        ctx.set_tuning(aca3d_waves=(1, 3, 4, 8))
    with pytest.raises(g.GcqError):
        ctx.set_tuning(aca3d_stack_slices=0)
    assert list(ctx.get_tuning().aca3d_waves) == [1, 1, 2, 4]
    assert ctx.get_tuning().aca3d_stack_slices == 2
    assert ctx.get_tuning().product_cols_per_wave == 32
    ctx.set_tuning(product_cols_per_wave=64)
    assert ctx.get_tuning().product_cols_per_wave == 64
    with pytest.raises(g.GcqError):
        ctx.set_tuning(product_cols_per_wave=48)
    assert ctx.get_tuning().product_cols_per_wave == 64


def test_rank_features_match_oracle_definition():
    """The rank model's pair features (host logic) against the oracle's
    definition, from the oracle tree's cluster boxes, for every far block and
    representative frequency."""
    from oracle import mlp
    from synth import freq
    xyz, tri = mesh.icosphere(3)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    ctx = g.Context(-1)
    ctx.upload_mesh(xyz, tri, 1.0)
    ctx.set_frequencies(s, True)
    ctx.build_cluster_tree(32, 1.0)
    _, T, B, _, _ = oracle_tree(xyz, tri, 32, 1.0)
    K = np.arange(len(s) // 2 + 1)
    far = [(a, b) for a, b, adm in B if adm]
    got = ctx.rank_features(K, len(far)).reshape(len(far), len(K), 5)
    lo, hi = np.array(T.bmin), np.array(T.bmax)
    for f, (a, b) in enumerate(far):
        diam = max(np.linalg.norm(hi[a] - lo[a]), np.linalg.norm(hi[b] - lo[b]))
        gap = np.maximum(0.0, np.maximum(lo[a] - hi[b], lo[b] - hi[a]))
        one = np.ones(len(K))
        ref = mlp.features(diam * one, np.linalg.norm(gap) * one, s[K], 1.0,
                           (T.end[a] - T.begin[a]) * one, (T.end[b] - T.begin[b]) * one)
        np.testing.assert_allclose(got[f], ref, rtol=1e-6, atol=1e-6)
    ctx.destroy()


def test_uploaded_oracle_tree_is_the_built_tree():
    """gcq_upload_cluster_tree with the oracle's partition gives the same
    partition, statistics and rank features as the library's own build."""
    from tests._oracle_tree_blocks import tree_arrays
    cfg = configs.get("housing3k")
    P, T, B, _, _ = oracle_tree(cfg["xyz"], cfg["tri"], 32, 1.0)
    a = g.Context(-1)
    a.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
    a.set_frequencies(cfg["s"])
    ia = a.build_cluster_tree(32, 1.0)
    b = g.Context(-1)
    b.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
    b.set_frequencies(cfg["s"])
    ib = b.upload_cluster_tree(*tree_arrays(T, B))
    for f in ("n_clusters", "n_leaves", "depth", "n_blocks", "n_far", "n_near", "far_dims",
              "near_entries"):
        assert getattr(ia, f) == getattr(ib, f), f
    pa, ba = a.get_tree()
    pb, bb = b.get_tree()
    assert np.array_equal(pa, pb) and np.array_equal(ba, bb)
    K = np.arange(0, 129, 16)
    assert np.array_equal(a.rank_features(K, ia.n_far), b.rank_features(K, ib.n_far))


def test_upload_cluster_tree_rejects_bad_partitions():
    from tests._oracle_tree_blocks import tree_arrays
    xyz, tri = mesh.icosphere(2)
    P, T, B, _, _ = oracle_tree(xyz, tri, 16, 1.0)
    ctx = g.Context(-1)
    with pytest.raises(g.GcqError):                      # no mesh yet
        ctx.upload_cluster_tree(*tree_arrays(T, B))
    ctx.upload_mesh(xyz, tri, 1.0)
    good = tree_arrays(T, B)
    ctx.upload_cluster_tree(*good)

    def bad(i, change):
        arrs = [x.copy() for x in good]
        change(arrs[i])
        with pytest.raises(g.GcqError):
            ctx.upload_cluster_tree(*arrs)

    def dup(p):
        p[1] = p[0]
    bad(0, dup)                                          # perm not a permutation
    bad(1, lambda cb: cb.__setitem__(0, 1))             # root not [0, n)
    son0 = int(np.nonzero(good[3][:, 0] >= 0)[0][0])

    def shift_son(s):
        s[son0, 0] = s[son0, 1]
    bad(3, shift_son)                                    # sons not distinct
    far = int(np.nonzero(good[6])[0][0])
    near = int(np.nonzero(good[6] == 0)[0][0])

    def drop(arr):
        arr[far] = arr[near]
    bad(4, drop)                                         # a repeated / missing pair
    bad(6, lambda a: a.__setitem__(near, 1) if True else None)   # touching boxes marked admissible
    # a block that overlaps others: the root pair added to the list
    arrs = [x.copy() for x in good]
    arrs[4] = np.append(arrs[4], 0).astype(np.int32)
    arrs[5] = np.append(arrs[5], 0).astype(np.int32)
    arrs[6] = np.append(arrs[6], 0).astype(np.uint8)
    with pytest.raises(g.GcqError):
        ctx.upload_cluster_tree(*arrs)
    # the context still holds the good tree
    perm, blocks = ctx.get_tree()
    assert np.array_equal(perm, good[0])
