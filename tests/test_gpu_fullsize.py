"""Parity at the benchmark's full sizes, in the configuration bench.py times,
on outputs the oracle computes one by one:

  * rows of the compressed per-frequency product (3D-ACA in complex64 at the
    workload's tolerance, float and split-bf16 products) of the 20480-triangle
    sphere (64 frequencies) and the 41520- and 77424-triangle housings (256
    frequencies) against dense float64 oracle rows: 64 sampled rows, the
    largest per-frequency relative error over 9 frequencies, 1e-5;
  * the timed per-frequency ACA (complex64 entries, recompression, tiles
    sized by the rank model) against the oracle's ACA on sampled (block,
    frequency) pairs of the sphere and the 41k housing;
  * the rank model trained on the spheres' ranks and used on the 77k housing:
    the same ranks and approximants as without it, and not slower.
"""
import numpy as np
import pytest
import torch

import paper_2505_00715_amd as g
from oracle import aca, entries
from oracle.geometry import Panels
from oracle.tree import ClusterTree, block_tree
from synth import configs, rhs
from tests._gpu_common import from_dev

pytestmark = pytest.mark.gpu

# ACA / 3D-ACA tolerance of each workload in bench.py (at 1e-5 the largest
# per-frequency error of the product exceeds 1e-5 on all three: 1.22e-5 at one
# frequency of the sphere, 1.18e-5 on the 77k housing, 9.4e-6 on the 41k one;
# the tolerance is tightened to 3e-6 as the reading of the tolerances
# prescribes), and the launch parameters its autotuner picks there (results
# depend on them only through the rounding order)
TOL = {"sphere20480": 3e-6, "housing40k": 3e-6, "housing80k": 3e-6}
TUNING = dict(aca3d_waves=(2, 4, 4, 4), aca3d_stack_slices=4, aca_waves=1)


def _ctx(cfg):
    ctx = g.Context(0)
    ctx.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
    ctx.set_frequencies(cfg["s"], True)
    ctx.build_cluster_tree(cfg["leaf"], cfg["eta"])
    ctx.set_tuning(**TUNING)
    return ctx


@pytest.mark.parametrize("name", ["sphere20480", "housing40k", "housing80k"])
def test_product_rows_per_frequency(name):
    cfg = configs.get(name)
    ctx = _ctx(cfg)
    st = ctx.aca3d(TOL[name], TOL[name], 40, g.C64)
    assert st.rank_max <= 40   # (n_capped also counts slices whose ACA reached its rank cap)
    L, n = len(cfg["s"]), len(cfg["tri"])
    X = rhs.random_complex(L, n, 0)
    Xd = torch.from_numpy(X).to(torch.complex64).cuda().reshape(-1)
    rows = rhs.sample_rows(n, 64, 0)
    kk = np.unique(np.linspace(0, L - 1, 9).round().astype(int))
    A = entries.block(Panels(cfg["xyz"], cfg["tri"]), rows, np.arange(n), cfg["s"][kk], cfg["c"])
    ref = np.einsum("kij,kj->ki", A, X[kk])
    for prec in (g.C64, g.C64_SPLIT_BF16):
        Yd = torch.zeros_like(Xd)
        ctx.compressed_matvec(g.PER_FREQUENCY, prec, Xd, Yd)
        Y = from_dev(Yd).reshape(L, n)
        per_k = np.linalg.norm(Y[kk][:, rows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
        print(f"{name} precision {prec}: per-frequency error max {per_k.max():.2e}")
        assert per_k.max() <= 1e-5, (prec, per_k)


def _rank_model(tol):
    """The rank model as bench.py trains it: the float64 plain ACA's ranks on
    the 320- and 20480-triangle spheres."""
    feats, targs = [], []
    for name in ("sphere320", "sphere20480"):
        cfg = configs.get(name)
        c = g.Context(0)
        c.upload_mesh(cfg["xyz"], cfg["tri"], cfg["c"])
        c.set_frequencies(cfg["s"], True)
        info = c.build_cluster_tree(cfg["leaf"], cfg["eta"])
        if info.n_far == 0:
            continue
        K = np.arange(len(cfg["s"]) // 2 + 1)
        c.aca_blocks(tol, 64, g.C128, g.FLAG_RECOMPRESS | g.FLAG_PER_FREQ_LAUNCH)
        feats.append(c.rank_features(K, info.n_far).reshape(-1, 5))
        targs.append(np.log1p(c.aca_ranks(len(K)).reshape(-1).astype(np.float32)))
    X, t = np.concatenate(feats), np.concatenate(targs)
    sel = np.random.default_rng(0).permutation(len(t))[:200000]
    m = g.Context(0)
    m.rank_model_train(X[sel], t[sel], epochs=40, batch=1024, lr=3e-3)
    return m.rank_model_get()


@pytest.fixture(scope="module")
def model():
    return _rank_model(3e-6)


@pytest.mark.parametrize("name", ["sphere20480", "housing40k"])
def test_timed_aca_path_matches_oracle(name, model):
    cfg = configs.get(name)
    tol = TOL[name]
    ctx = _ctx(cfg)
    ctx.rank_model_set(*model)
    K = np.arange(len(cfg["s"]) // 2 + 1)
    fr = K[[0, len(K) // 2, len(K) - 1]]
    ctx.aca_blocks(tol, 64, g.C64, g.FLAG_RECOMPRESS | g.FLAG_USE_PREDICTOR, freq_idx=fr)
    P = Panels(cfg["xyz"], cfg["tri"])
    T = ClusterTree(P, cfg["leaf"])
    B = block_tree(T, cfg["eta"])
    far = [b for b, (_, _, adm) in enumerate(B) if adm]
    rng = np.random.default_rng(1)
    num = den = num_t = num_o = 0.0
    for b in rng.choice(far, 30, replace=False):
        I, J = T.indices(B[b][0]), T.indices(B[b][1])
        for k in fr:
            A = entries.block(P, I, J, [cfg["s"][k]], cfg["c"])[0]
            Uo, Vo, _ = aca.aca_block(P, I, J, cfg["s"][k], cfg["c"], tol, 64, recompress_tol=tol)
            Ug, Vg = ctx.get_block_factors(int(b), int(k))
            Sg, So = Ug @ Vg.conj().T, Uo @ Vo.conj().T
            num += np.linalg.norm(Sg - So) ** 2
            num_t += np.linalg.norm(Sg - A) ** 2
            num_o += np.linalg.norm(So - A) ** 2
            den += np.linalg.norm(A) ** 2
            assert np.linalg.norm(Sg - A) <= 40 * tol * np.linalg.norm(A) + 1e-30
    assert np.sqrt(num / den) <= 1e-4
    # the complex64 path's error against the dense blocks: the oracle's own
    # ACA error (float rounding of the entries adds up to ~1e-6)
    assert np.sqrt(num_t / den) <= 1.5 * np.sqrt(num_o / den) + 2e-6


def test_rank_model_gain_on_the_80k_housing(model):
    """Trained on the spheres, used on the 77k housing: the ranks and the
    approximants are those of the run without the model, and the run is
    not slower (bench.py reports both times)."""
    import time
    cfg = configs.get("housing80k")
    tol = TOL["housing80k"]
    ctx = _ctx(cfg)
    ctx.rank_model_set(*model)
    K = np.arange(len(cfg["s"]) // 2 + 1)
    fr = K[::32]
    ms = {}
    ranks, facs = {}, {}
    blocks = ctx.get_tree()[1]
    far = np.nonzero(blocks[:, 4])[0]
    pick = np.random.default_rng(2).choice(far, 12, replace=False)
    for flags in (g.FLAG_RECOMPRESS | g.FLAG_USE_PREDICTOR, g.FLAG_RECOMPRESS):
        ctx.aca_blocks(tol, 64, g.C64, flags, freq_idx=fr)            # warm-up
        st = ctx.aca_blocks(tol, 64, g.C64, flags, freq_idx=fr)
        ms[flags] = st.device_ms
        ranks[flags] = ctx.aca_ranks(len(fr))
        facs[flags] = [ctx.get_block_factors(int(b), int(fr[1])) for b in pick]
    with_p, without = g.FLAG_RECOMPRESS | g.FLAG_USE_PREDICTOR, g.FLAG_RECOMPRESS
    print(f"aca_blocks on {len(fr)} frequencies: {ms[without]:.1f} ms without the model, "
          f"{ms[with_p]:.1f} ms with it")
    assert np.array_equal(ranks[with_p], ranks[without])
    for (Ua, Va), (Ub, Vb) in zip(facs[with_p], facs[without]):
        Sa, Sb = Ua @ Va.conj().T, Ub @ Vb.conj().T
        assert np.linalg.norm(Sa - Sb) <= 1e-6 * np.linalg.norm(Sb)
    assert ms[with_p] <= ms[without]
