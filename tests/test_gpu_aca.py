"""GPU parity of the per-frequency ACA with recompression (gcq_aca_blocks) and
of the per-frequency H-matrix product, against the oracle's ACA on the same
blocks: approximants (not factors, since different pivots give different but
equally valid factors) and products, in complex128 and complex64."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import aca, entries, matvec
from oracle.geometry import Panels
from synth import freq, mesh, rhs
from tests._gpu_common import from_dev, kpos_map, make_ctx, rel, to_dev
from tests._oracle_tree_blocks import oracle_tree

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _problem():
    xyz, tri = mesh.icosphere(3)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    return xyz, tri, s


@pytest.mark.parametrize("prec,waves", [(g.C128, 1), (g.C64, 1), (g.C128, 2), (g.C64, 4)])
def test_aca_blocks_match_oracle(prec, waves):
    """Also with 2 and 4 waves per (block, frequency) pair."""
    xyz, tri, s = _problem()
    P, T, B, perm, blocks = oracle_tree(xyz, tri, 32, 1.0)
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.set_tuning(aca_waves=waves)
    st = ctx.aca_blocks(TOL, 64, prec, g.FLAG_RECOMPRESS)
    rep, conj, K, kpos = kpos_map(s)
    assert st.n_pairs == int(blocks[:, 4].sum()) * len(K)
    far = np.nonzero(blocks[:, 4])[0]
    rng = np.random.default_rng(0)
    num = den = num_t = num_o = 0.0
    same_rank = total = 0
    for b in rng.choice(far, 40, replace=False):
        a, bb = B[b][0], B[b][1]
        I, J = T.indices(a), T.indices(bb)
        for k in K[:: 2]:
            A = entries.block(P, I, J, [s[k]], 1.0)[0]
            Uo, Vo, info = aca.aca_block(P, I, J, s[k], 1.0, TOL, 64, recompress_tol=TOL)
            Ug, Vg = ctx.get_block_factors(int(b), int(k))
            Sg, So = Ug @ Vg.conj().T, Uo @ Vo.conj().T
            num += np.linalg.norm(Sg - So) ** 2
            num_t += np.linalg.norm(Sg - A) ** 2
            num_o += np.linalg.norm(So - A) ** 2
            den += np.linalg.norm(A) ** 2
            same_rank += Ug.shape[1] == Uo.shape[1]
            total += 1
            # every block stays within the ACA's own error regime
            assert np.linalg.norm(Sg - A) <= 40 * TOL * np.linalg.norm(A) + 1e-30
    assert np.sqrt(num / den) <= (1e-5 if prec == g.C128 else 1e-4)
    # approximation error against the dense blocks: that of the oracle's ACA
    assert np.sqrt(num_t / den) <= 1.5 * np.sqrt(num_o / den) + 1e-6
    if prec == g.C128:
        assert same_rank >= 0.8 * total


def test_recompression_rank_classes():
    """At ACA tolerance 1e-10 the ACA ranks of the 1280-triangle sphere's far
    blocks reach past 32, so every rank class of the recompression runs
    (LDS matrices sized for ranks up to 8, 12, 16, 18, 24, 32 with one to four
    waves per pair, global scratch above): the approximants of the largest
    blocks and of random ones hold the tolerance against the dense blocks and
    agree with the oracle's ACA with recompression."""
    xyz, tri, s = _problem()
    tol = 1e-10
    P, T, B, perm, blocks = oracle_tree(xyz, tri, 32, 1.0)
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    st = ctx.aca_blocks(tol, 64, g.C128, g.FLAG_RECOMPRESS)
    assert st.status == g.OK
    rep, conj, K, kpos = kpos_map(s)
    r = ctx.aca_ranks(len(K))
    # recompressed ranks bound the ACA ranks from below: classes above 18, 24, 32 ran
    assert r.max() > 32 and ((r > 18) & (r <= 24)).any() and ((r > 24) & (r <= 32)).any()
    far = np.nonzero(blocks[:, 4])[0]
    big = sorted(far, key=lambda b: -(len(T.indices(B[b][0])) + len(T.indices(B[b][1]))))[:8]
    rng = np.random.default_rng(2)
    pick = list(big) + list(rng.choice(far, 8, replace=False))
    num = den = 0.0
    for b in pick:
        I, J = T.indices(B[b][0]), T.indices(B[b][1])
        for k in (K[0], K[len(K) // 2], K[-1]):
            A = entries.block(P, I, J, [s[k]], 1.0)[0]
            Ug, Vg = ctx.get_block_factors(int(b), int(k))
            Sg = Ug @ Vg.conj().T
            assert np.linalg.norm(Sg - A) <= 40 * tol * np.linalg.norm(A) + 1e-30, (b, k)
            Uo, Vo, _ = aca.aca_block(P, I, J, s[k], 1.0, tol, 64, recompress_tol=tol)
            num += np.linalg.norm(Sg - Uo @ Vo.conj().T) ** 2
            den += np.linalg.norm(A) ** 2
    assert np.sqrt(num / den) <= 40 * tol


@pytest.mark.parametrize("prec", [g.C128, g.C64])
def test_plain_h_product(prec):
    xyz, tri, s = _problem()
    P, T, B, perm, blocks = oracle_tree(xyz, tri, 32, 1.0)
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    ctx.aca_blocks(TOL, 64, prec, g.FLAG_RECOMPRESS)
    rep, conj, K, kpos = kpos_map(s)
    X = rhs.random_complex(len(s), P.n, 0)
    Y = torch.zeros(len(s) * P.n, dtype=torch.complex128 if prec == g.C128 else torch.complex64,
                    device="cuda")
    ctx.compressed_matvec(g.PLAIN_H, prec, to_dev(X, prec).reshape(-1), Y)
    Yg = from_dev(Y).reshape(len(s), P.n)
    # oracle H-matrix from the oracle's own ACA
    hb = []
    for a, bb, adm in B:
        I, J = T.indices(a), T.indices(bb)
        data = {}
        for k in K:
            if adm:
                U, V, _ = aca.aca_block(P, I, J, s[k], 1.0, TOL, 64, recompress_tol=TOL)
                data[k] = (U, V)
            else:
                data[k] = entries.block(P, I, J, [s[k]], 1.0)[0]
        hb.append((I, J, adm, data))
    Yo = matvec.hmatrix(hb, X, rep, conj)
    err = rel(Yg, Yo)
    assert err <= (1e-5 if prec == g.C128 else 1e-4), err
    # and against the dense operator
    Yt = matvec.dense(entries.dense(P, s, 1.0), X)
    assert rel(Yg, Yt) <= 1e-5


def test_aca_per_frequency_launch_baseline_equals_batched():
    xyz, tri, s = _problem()
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    st1 = ctx.aca_blocks(TOL, 64, g.C128, g.FLAG_RECOMPRESS | g.FLAG_PER_FREQ_LAUNCH)
    f1 = ctx.get_block_factors(int(np.nonzero(ctx.get_tree()[1][:, 4])[0][3]), 0)
    st2 = ctx.aca_blocks(TOL, 64, g.C128, g.FLAG_RECOMPRESS)
    f2 = ctx.get_block_factors(int(np.nonzero(ctx.get_tree()[1][:, 4])[0][3]), 0)
    assert st1.rank_sum == st2.rank_sum and st1.n_pairs == st2.n_pairs
    assert np.array_equal(f1[0], f2[0]) and np.array_equal(f1[1], f2[1])


def test_aca_without_recompression_and_rank_cap():
    xyz, tri, s = _problem()
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    st = ctx.aca_blocks(TOL, 64, g.C128, 0)
    assert st.rank_sum == st.aca_rank_sum
    st2 = ctx.aca_blocks(TOL, 64, g.C128, g.FLAG_RECOMPRESS)
    assert st2.rank_sum < st.rank_sum and st2.aca_rank_sum == st.aca_rank_sum
    st3 = ctx.aca_blocks(1e-12, 3, g.C128, 0)
    assert st3.n_capped > 0 and st3.rank_max == 3 and st3.status == g.RANK_CAPPED
    with pytest.raises(g.GcqError):
        ctx.aca_blocks(TOL, 65, g.C128, 0)
