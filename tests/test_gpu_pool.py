"""Parity of the pair pool (Sec. IV-C, the Augmented-Pair variant: walk pairs collected
before training, training pairs drawn from their recombinations) on the GPU with the
oracle, through the C ABI.

Integer work (the collected pairs and every sampled tuple) must match bit for bit, at
indices past 2^32 and 2^41, for the smallest and the largest pools the buffer holds and
for C2's pool at its training size; SNAPSHOT training on pool pairs must agree with the
binary64 oracle within 1e-5 relative error per row; Hogwild training on pool pairs must
match the oracle's held-out AUC within 0.005.
"""
import json
import os

import numpy as np
import pytest

import oracle
from synth import config_graph

from gpu_util import dot_rows, max_row_rel_err, trainer_for

pytestmark = pytest.mark.gpu
WALK = dict(L=100, W=2, Bw=1024)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TUNE_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2604_09419_amd",
                          "tune_cache.json")


def _lh():
    import paper_2604_09419_amd as lh
    return lh


def _oracle_walk(g, L, W, Bw):
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    return t, oracle.WalkGraph(t, L=L, W=W, Bw=Bw)


def _tuples_equal(tr, t, wg, seed, gid, K, R, first, count):
    u, v, neg = tr.sample(first, count)
    _, _, ou, ov = wg.pool(seed=seed, graph_id=gid, R=R, first=first, count=count)
    oneg = oracle.sample_negatives(t.n, t.nthr, t.nalias, seed=seed, graph_id=gid, K=K, first=first, count=count)
    assert np.array_equal(u.cpu().numpy(), ou), (R, first)
    assert np.array_equal(v.cpu().numpy(), ov), (R, first)
    assert np.array_equal(neg.cpu().numpy(), oneg), (R, first)


@pytest.mark.parametrize("L,W,Bw", [(100, 2, 1024), (7, 3, 5)])
def test_pool_tuples_bitwise(L, W, Bw):
    g, _, _, _ = config_graph("C1")
    tr = trainer_for(g, d=8, K=3, orders=2, seed=9, total_samples=1_000_000, graph_id=3, init=False)
    tr.build_walks(walk_length=L, window=W, walks_per_batch=Bw)
    t, wg = _oracle_walk(g, L, W, Bw)
    for R in (1, 2, 1415, Bw * wg.pairs_per_walk + 3):
        print(f"pool L={L} W={W} Bw={Bw} R={R}", flush=True)
        tr.build_pool(R)
        for first, count in [(0, 100_003), (2**33 + 7, 50_000), (2**41 + 5, 4097)]:
            _tuples_equal(tr, t, wg, 9, 3, 3, R, first, count)
    # back to the walk pairs
    tr.drop_pool()
    u, v = tr.walk_pairs(5, 20_000)
    ou, ov = wg.pairs(seed=9, graph_id=3, first=5, count=20_000)
    assert np.array_equal(u.cpu().numpy(), ou) and np.array_equal(v.cpu().numpy(), ov)
    tr.close()


def test_pool_default_size_and_limits():
    """The default pool for T samples is the oracle's size; the largest pool is the pair
    buffer (whole walk batches of about 2^24 pairs), one more is refused; lh_walk_pairs is
    refused while a pool is on; rebuilding the walks ends the pool."""
    lh = _lh()
    g, _, _, _ = config_graph("C1")
    T = 10**6
    tr = trainer_for(g, d=8, K=2, orders=2, seed=4, total_samples=T, init=False)
    with pytest.raises(lh._lib.LhError):
        tr.build_pool(10)  # no walks yet
    tr.build_walks(walk_length=100, window=2, walks_per_batch=1024)
    assert tr.build_pool() == oracle.pool_size(T)
    with pytest.raises(lh._lib.LhError):
        tr.walk_pairs(0, 10)
    cap = 1024 * 99 * ((1 << 24) // (1024 * 99))
    t, wg = _oracle_walk(g, 100, 2, 1024)
    tr.build_pool(cap)
    for first, count in [(0, 30_000), (2**40 + 1, 30_000)]:
        _tuples_equal(tr, t, wg, 4, 0, 2, cap, first, count)
    with pytest.raises(lh._lib.LhError):
        tr.build_pool(cap + 1)
    tr.build_walks(walk_length=100, window=2, walks_per_batch=1024)
    u, v = tr.walk_pairs(0, 1000)
    ou, ov = wg.pairs(seed=4, graph_id=0, first=0, count=1000)
    assert np.array_equal(u.cpu().numpy(), ou) and np.array_equal(v.cpu().numpy(), ov)
    tr.close()


def test_pool_tuples_c2_at_training_size():
    """C2 with the pool its training run uses (T = 2e8: R = 20,001), in the tile shape the
    bench times: tuples at sampled positions over the whole run."""
    from synth import CONFIGS
    cfg = CONFIGS["C2"]
    g, _, _, _ = config_graph("C2", holdout=True)
    tr = trainer_for(g, d=cfg["d"], K=cfg["K"], orders=3, seed=cfg["seed"], total_samples=cfg["T"], init=False)
    tr.build_walks(walk_length=WALK["L"], window=WALK["W"], walks_per_batch=WALK["Bw"])
    R = tr.build_pool()
    assert R == oracle.pool_size(cfg["T"]) == 20_001
    t, wg = _oracle_walk(g, **WALK)
    for first in (0, 77_777_777, cfg["T"] - 65_536):
        print(f"C2 pool tuples at {first}", flush=True)
        _tuples_equal(tr, t, wg, cfg["seed"], 0, cfg["K"], R, first, 65_536)
    tr.close()


@pytest.mark.parametrize("B,orders,K", [(1024, 2, 5), (99, 3, 1)])
def test_pool_snapshot_c1_within_1e5(B, orders, K):
    lh = _lh()
    g, _, _, _ = config_graph("C1")
    t, wg = _oracle_walk(g, **WALK)
    T, count = 1_000_000, 250_000
    R = oracle.pool_size(T)
    tr = trainer_for(g, d=16, K=K, orders=orders, seed=1, total_samples=T, mode="snapshot", batch=B, lam=0.01,
                     alpha_neg=0.8)
    tr.build_walks(walk_length=WALK["L"], window=WALK["W"], walks_per_batch=WALK["Bw"])
    tr.build_pool(R)
    m = oracle.Model(t, d=16, K=K, orders=orders, T=T, seed=1, lam=0.01, alpha=0.8)
    tr.train_steps(0, count)
    m.train(0, count, "snapshot", B, walks=wg, pool=R)
    tr.check()
    for name, tab, ref in (("U", lh.LH_TABLE_U, m.U), ("C", lh.LH_TABLE_C, m.C), ("U1", lh.LH_TABLE_U1, m.U1)):
        if ref is None:
            continue
        err = max_row_rel_err(tr.read(tab).cpu().numpy(), ref)
        print(f"pool snapshot B={B} orders={orders} K={K} {name}: max row rel err {err:.3e}", flush=True)
        assert err <= 1e-5, (name, err)
    tr.close()


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_pool_hogwild_c1_auc_matches_oracle(dtype):
    """Hogwild on pool pairs against the oracle's SEQ run on the same pool (with bfloat16
    storage for bf16 tables): held-out AUCs within 0.005."""
    from synth import CONFIGS
    lh = _lh()
    cfg = CONFIGS["C1"]
    g, hs, hd, neg = config_graph("C1", holdout=True)
    t, wg = _oracle_walk(g, **WALK)
    R = oracle.pool_size(cfg["T"])
    m = oracle.Model(t, d=16, K=5, orders=2, T=cfg["T"], seed=cfg["seed"], eta0=cfg["eta0"],
                     storage="bf16" if dtype == "bf16" else "binary64")
    m.train(0, cfg["T"], "seq", walks=wg, pool=R)
    ref = (oracle.auc(m.scores(hs, hd, 2), m.scores(hs, neg, 2)),
           oracle.auc(oracle.pair_scores(m.U, m.U, hs, hd), oracle.pair_scores(m.U, m.U, hs, neg)))
    tr = trainer_for(g, d=16, K=5, orders=2, dtype=dtype, seed=cfg["seed"], total_samples=cfg["T"])
    tr.build_walks(walk_length=WALK["L"], window=WALK["W"], walks_per_batch=WALK["Bw"])
    tr.build_pool()
    tr.train_steps(0, cfg["T"])
    tr.check()
    U = tr.read(lh.LH_TABLE_U).cpu().numpy()
    C = tr.read(lh.LH_TABLE_C).cpu().numpy()
    got = (oracle.auc(dot_rows(U, C, hs, hd), dot_rows(U, C, hs, neg)),
           oracle.auc(dot_rows(U, U, hs, hd), dot_rows(U, U, hs, neg)))
    print(f"C1 pool {dtype}: uc {got[0]:.4f} (oracle {ref[0]:.4f}) uu {got[1]:.4f} (oracle {ref[1]:.4f})", flush=True)
    assert abs(got[0] - ref[0]) <= 0.005 and abs(got[1] - ref[1]) <= 0.005
    tr.close()


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "c2_pool_oracle_auc.json")),
                    reason="stored reference not written yet (make_golden.py c2_pool_auc)")
@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_pool_hogwild_c2_auc_matches_oracle(dtype):
    """C2 (orders 1+2, T = 2e8) on its pool of 20,001 pairs, in the tile shape the bench
    times: every held-out AUC within 0.005 of the oracle's SEQ binary64 run."""
    from synth import CONFIGS
    lh = _lh()
    gold = json.load(open(os.path.join(GOLDEN, "c2_pool_oracle_auc.json")))
    cfg = CONFIGS["C2"]
    g, hs, hd, neg = config_graph("C2", holdout=True)
    assert (g.n, g.m, hs.size) == (gold["n"], gold["m_train"], gold["held_out"])
    tr = trainer_for(g, d=cfg["d"], K=cfg["K"], orders=3, dtype=dtype, seed=cfg["seed"], total_samples=cfg["T"])
    tr.tune(probe=20_000_000, cache_path=TUNE_CACHE)
    tr.build_walks(walk_length=WALK["L"], window=WALK["W"], walks_per_batch=WALK["Bw"])
    tr.build_pool()
    tr.train_steps(0, cfg["T"])
    tr.check()
    U = tr.read(lh.LH_TABLE_U).cpu().numpy()
    C = tr.read(lh.LH_TABLE_C).cpu().numpy()
    U1 = tr.read(lh.LH_TABLE_U1).cpu().numpy()
    uu = (dot_rows(U, U, hs, hd), dot_rows(U, U, hs, neg))
    o1 = (dot_rows(U1, U1, hs, hd), dot_rows(U1, U1, hs, neg))
    got = {"uc": oracle.auc(dot_rows(U, C, hs, hd), dot_rows(U, C, hs, neg)), "uu": oracle.auc(*uu),
           "o1": oracle.auc(*o1), "concat": oracle.auc(uu[0] + o1[0], uu[1] + o1[1])}
    for k, v in got.items():
        print(f"C2 pool {dtype} {k}: {v:.4f} (oracle {gold['auc_' + k]:.4f})", flush=True)
    for k, v in got.items():
        assert abs(v - gold["auc_" + k]) <= 0.005, k
    tr.close()
