"""GPU parity of the batched GMRES solve and of the rank-prediction network
(forward, backward against the oracle's float64 back-propagation, training),
and the predictor ablation: sizing tiles from the network changes neither the
ranks nor the factors the adaptive ACA produces."""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import aca3d, entries, matvec, mlp
from oracle.geometry import Panels
from synth import freq, mesh, rhs
from tests._gpu_common import from_dev, kpos_map, make_ctx, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,rtol", [(g.C128, 1e-9), (g.C64, 1e-6), (g.C64_SPLIT_BF16, 1e-6)])
def test_gmres_all_frequencies(prec, rtol):
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(8, 0.05, 1e-8 ** (1 / 8))
    ctx = make_ctx(xyz, tri, 1.0, s, 16, 1.0)
    # split-bf16 products apply an operator built in complex64
    ctx.aca3d(1e-10, 1e-10, 40, g.C64 if prec == g.C64_SPLIT_BF16 else prec)
    Bh = rhs.random_complex(len(s), 320, 1)
    B = to_dev(Bh, g.C128).reshape(-1)
    X = torch.zeros_like(B)
    st = ctx.solve(B, X, rtol=rtol, max_iter=400, restart=30, precision=prec)
    assert st.status == g.OK and st.n_converged == len(s)
    x = from_dev(X).reshape(len(s), 320)
    P = Panels(xyz, tri)
    A = entries.dense(P, s, 1.0)
    for k in range(len(s)):
        xs = np.linalg.solve(A[k], Bh[k])
        # 3D-ACA tolerance 1e-10 and the GMRES tolerance bound the difference
        assert rel(x[k], xs) <= 1e3 * max(rtol, 1e-10) * 10
        res = np.linalg.norm(A[k] @ x[k] - Bh[k]) / np.linalg.norm(Bh[k])
        # split-bf16 solves with the operator's two-plane copy, a fixed relative
        # perturbation of at most 2^-18 per entry: its residual against A holds
        # that perturbation times |A| |x| / |b| on top of rtol
        pert = 0.0 if prec != g.C64_SPLIT_BF16 else \
            2.0 ** -18 * np.linalg.norm(np.abs(A[k]), 2) * np.linalg.norm(x[k]) / np.linalg.norm(Bh[k])
        assert res <= 2 * rtol + 1e-8 + pert, (res, pert)


@pytest.mark.parametrize("prec", [g.C128, g.C64, g.C64_SPLIT_BF16])
def test_gmres_graph_step_matches_host_path(prec):
    """The device-side Arnoldi step replayed as a graph (default) against the
    host's least-squares path (graphs off): both converge in the same number
    of iterations (restart 6: several restart cycles and graph replays per
    cycle) to the same solutions, and the graph solve repeated gives the
    same result again (to rounding where the product's sums are ordered by
    atomics)."""
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(8, 0.05, 1e-8 ** (1 / 8))
    ctx = make_ctx(xyz, tri, 1.0, s, 16, 1.0)
    ctx.aca3d(1e-10, 1e-10, 40, g.C64 if prec == g.C64_SPLIT_BF16 else prec)
    rtol = 1e-9 if prec == g.C128 else 1e-6      # complex64 products: float rounding
    B = to_dev(rhs.random_complex(len(s), 320, 2), g.C128).reshape(-1)
    out = {}
    for graph in (1, 0, 1):
        ctx.set_tuning(product_graph=graph)
        X = torch.zeros_like(B)
        st = ctx.solve(B, X, rtol=rtol, max_iter=200, restart=6, precision=prec)
        assert st.status == g.OK and st.n_converged == len(s)
        out.setdefault(graph, []).append((st.iters_max, from_dev(X).reshape(len(s), 320)))
    (ig, xg), (ig2, xg2) = out[1]
    ih, xh = out[0][0]
    assert abs(ig - ih) <= 1, (ig, ih)
    assert rel(xg, xh) <= 100 * rtol
    # the float product adds its blocks with atomics (order-dependent rounding)
    assert ig2 == ig and rel(xg2, xg) <= (1e-12 if prec == g.C128 else 10 * rtol)


@pytest.mark.parametrize("prec", [g.C64_SPLIT_BF16, g.C64])
def test_gmres_converged_tiles_left_out(prec):
    """96 frequencies (three 32-column tiles; the middle one, of large |s|,
    converges first): the graph path leaves a tile whose systems have all
    converged out of the split-bf16 product and back-substitutes each system
    over the steps its tile computed; the host path computes every product and
    applies the same rule. Both give the same iterations and solutions, every
    system converges, and sampled systems hold the tolerance against the
    dense oracle matrix."""
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(96, 0.05, 1e-8 ** (1 / 48))
    L = len(s)
    assert L == 96
    ctx = make_ctx(xyz, tri, 1.0, s, 16, 1.0)
    ctx.aca3d(1e-8, 1e-8, 40, g.C64)
    rtol = 1e-6
    Bh = rhs.random_complex(L, 320, 3)
    B = to_dev(Bh, g.C128).reshape(-1)
    out = {}
    for graph in (1, 0):
        ctx.set_tuning(product_graph=graph)
        X = torch.zeros_like(B)
        st = ctx.solve(B, X, rtol=rtol, max_iter=300, restart=20, precision=prec)
        assert st.status == g.OK and st.n_converged == L
        out[graph] = (st.iters_max, from_dev(X).reshape(L, 320))
    ctx.set_tuning(product_graph=1)
    (ig, xg), (ih, xh) = out[1], out[0]
    assert abs(ig - ih) <= 1, (ig, ih)
    assert rel(xg, xh) <= 100 * rtol
    kk = np.array([0, 31, 40, 55, 70, 95])
    A = entries.dense(Panels(xyz, tri), s[kk], 1.0)
    for a, k in zip(A, kk):
        res = np.linalg.norm(a @ xg[k] - Bh[k]) / np.linalg.norm(Bh[k])
        pert = 0.0 if prec != g.C64_SPLIT_BF16 else \
            2.0 ** -18 * np.linalg.norm(np.abs(a), 2) * np.linalg.norm(xg[k]) / np.linalg.norm(Bh[k])
        # 3D-ACA tolerance 1e-8 and float products on top of rtol
        assert res <= 3 * rtol + 1e-7 + pert, (k, res, pert)


def test_gmres_not_converged_flag():
    xyz, tri = mesh.icosphere(2)
    s = freq.bdf2_circle(8, 0.05, 1e-8 ** (1 / 8))
    ctx = make_ctx(xyz, tri, 1.0, s, 16, 1.0)
    ctx.aca3d(1e-8, 1e-8, 40, g.C128)
    B = to_dev(rhs.random_complex(len(s), 320, 1), g.C128).reshape(-1)
    X = torch.zeros_like(B)
    st = ctx.solve(B, X, rtol=1e-14, max_iter=3, restart=30, precision=g.C128)
    assert st.status == g.NOT_CONVERGED and st.n_converged < len(s)


def _samples(m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, 5))
    t = np.log1p(np.abs(3 + 2 * X[:, 0] - X[:, 1] + 0.5 * X[:, 3] * X[:, 4]))
    return X, t


def test_mlp_forward_backward_vs_oracle():
    ctx = g.Context(0)
    theta = mlp.glorot_init(7)
    ctx.rank_model_set(theta.astype(np.float32), np.zeros(5, np.float32), np.ones(5, np.float32))
    X, t = _samples(300, 3)
    loss, grad = ctx.rank_model_grad(X.astype(np.float32), t.astype(np.float32))
    th32 = theta.astype(np.float32).astype(np.float64)
    lo, go = mlp.loss_and_grad(th32, X.astype(np.float32).astype(np.float64),
                               t.astype(np.float32).astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    assert np.linalg.norm(grad - go) <= 1e-4 * np.linalg.norm(go)
    pred = ctx.rank_model_predict(X.astype(np.float32))
    yo, _ = mlp.forward(th32, X.astype(np.float32).astype(np.float64))
    assert np.abs(pred - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())


def test_mlp_training_reduces_loss():
    # 100 epochs: the float64 oracle's own Adam training on these samples ends
    # at 0.115-0.144 var(t) after 40 epochs (seeds 0-2), at 0.020-0.030 after 100
    ctx = g.Context(0)
    X, t = _samples(4096, 5)
    st = ctx.rank_model_train(X.astype(np.float32), t.astype(np.float32), epochs=100, batch=256,
                              lr=3e-3)
    assert st.loss_last < 0.2 * st.loss_first
    pred = ctx.rank_model_predict(X.astype(np.float32))
    assert np.mean((pred - t) ** 2) < 0.1 * np.var(t) + 1e-3


def test_predictor_ablation_same_result():
    xyz, tri = mesh.icosphere(3)
    s = freq.bdf2_circle(16, 0.05, 1e-8 ** (1 / 16))
    ctx = make_ctx(xyz, tri, 1.0, s, 32, 1.0)
    rep, conj, K, kpos = kpos_map(s)
    st0 = ctx.aca_blocks(1e-5, 64, g.C128, g.FLAG_RECOMPRESS)
    far = np.nonzero(ctx.get_tree()[1][:, 4])[0]
    ranks0 = [ctx.get_block_factors(int(b), int(k))[0].shape[1] for b in far for k in K]
    # training data: ranks of the plain ACA
    feat = ctx.rank_features(K, len(far)).reshape(-1, 5)
    targ = np.log1p(np.array(ranks0, np.float32).reshape(len(far), len(K)).reshape(-1))
    tr = ctx.rank_model_train(feat, targ, epochs=60, batch=512, lr=3e-3)
    assert tr.loss_last < tr.loss_first
    X = to_dev(rhs.random_complex(len(s), 1280, 0), g.C128).reshape(-1)
    Y0 = torch.zeros_like(X)
    ctx.compressed_matvec(g.PLAIN_H, g.C128, X, Y0)
    y0 = from_dev(Y0)
    st1 = ctx.aca_blocks(1e-5, 64, g.C128, g.FLAG_RECOMPRESS | g.FLAG_USE_PREDICTOR)
    ranks1 = [ctx.get_block_factors(int(b), int(k))[0].shape[1] for b in far for k in K]
    assert ranks0 == ranks1
    assert st1.rank_sum == st0.rank_sum and st1.aca_rank_sum == st0.aca_rank_sum
    Y1 = torch.zeros_like(X)
    ctx.compressed_matvec(g.PLAIN_H, g.C128, X, Y1)
    y1 = from_dev(Y1)
    assert rel(y1, y0) <= 1e-13   # same factors; only the order of atomic sums differs
    # a model predicting rank 0 forces every pair through the overflow path
    ctx.rank_model_set(np.zeros(g.N_MODEL_PARAMS, np.float32))
    st2 = ctx.aca_blocks(1e-5, 64, g.C128, g.FLAG_RECOMPRESS | g.FLAG_USE_PREDICTOR)
    assert st2.n_overflow > 0 and st2.rank_sum == st0.rank_sum
