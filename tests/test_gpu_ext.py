"""The two extensions on the GPU: bfloat16 tables with stochastic rounding, and many
graphs trained in one persistent, hipGraph-captured launch.  Also the tuner's dry runs."""
import json
import os

import numpy as np
import pytest

import oracle
from synth import config_graph, rmat_graph, small_batch

from gpu_util import dot_rows, fro_rel_err, max_row_rel_err, trainer_for

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lh():
    import paper_2604_09419_amd as lh
    return lh


def _auc_uc_uu(tr, hs, hd, neg):
    lh = _lh()
    U = tr.read(lh.LH_TABLE_U).cpu().numpy()
    C = tr.read(lh.LH_TABLE_C).cpu().numpy()
    return (oracle.auc(dot_rows(U, C, hs, hd), dot_rows(U, C, hs, neg)),
            oracle.auc(dot_rows(U, U, hs, hd), dot_rows(U, U, hs, neg)))


@pytest.mark.parametrize("hot_shadow", [False, True])
def test_bf16_hogwild_c1_auc_matches_oracle(hot_shadow):
    """C1's tables fit in one L2, so every touched row is hot: this exercises the hot-row
    write path alone (packed bfloat16 atomics, or the binary32 shadow)."""
    gold = json.load(open(os.path.join(GOLDEN, "c1_oracle_auc.json")))
    g, hs, hd, neg = config_graph("C1", holdout=True)
    tr = trainer_for(g, d=16, K=5, orders=2, dtype="bf16", seed=gold["seed"], total_samples=gold["T"],
                     hot_shadow=hot_shadow)
    tr.train_steps(0, gold["T"])
    tr.check()
    uc, uu = _auc_uc_uu(tr, hs, hd, neg)
    print(f"C1 bf16 hogwild{' shadow' if hot_shadow else ''} AUC uc {uc:.4f} (oracle {gold['auc_uc']:.4f}) uu {uu:.4f} "
          f"(oracle {gold['auc_uu']:.4f})", flush=True)
    assert abs(uc - gold["auc_uc"]) <= 0.005 and abs(uu - gold["auc_uu"]) <= 0.005


def test_bf16_zero_step_leaves_tables_bitwise():
    """With eta0 = 0 every written value is already bfloat16, and stochastic rounding of an
    exactly representable value returns it unchanged (hot rows: a zero increment)."""
    lh = _lh()
    g = rmat_graph(12, 3000, 30_000, seed=3)
    for mode, shadow in (("hogwild", False), ("hogwild", True), ("snapshot", False)):
        tr = trainer_for(g, d=64, K=5, orders=3, dtype="bf16", eta0=0.0, seed=4, total_samples=100_000,
                         mode=mode, batch=4096, hot_shadow=shadow)
        before = [tr.read(t).cpu().numpy() for t in (0, 1, 2)]
        tr.train_steps(0, 100_000 if mode == "hogwild" else 4096 * 10)
        tr.check()
        after = [tr.read(t).cpu().numpy() for t in (0, 1, 2)]
        for x, y in zip(before, after):
            assert np.array_equal(x, y)


def test_bf16_snapshot_embedding_error_is_small(c1_graph, c1_tables):
    lh = _lh()
    T, B = 1_000_000, 256
    tr = trainer_for(c1_graph, d=16, K=5, orders=2, dtype="bf16", seed=1, total_samples=T, mode="snapshot",
                     batch=B)
    tr.train_steps(0, T)
    m = oracle.Model(c1_tables, d=16, K=5, orders=2, T=T, seed=1)
    m.train(0, T, "snapshot", B)
    for tab, ref in ((lh.LH_TABLE_U, m.U), (lh.LH_TABLE_C, m.C)):
        err = fro_rel_err(tr.read(tab).cpu().numpy(), ref)
        print(f"C1 bf16 SNAPSHOT B={B} table {tab}: embedding error {err:.3e}", flush=True)
        # Each stochastic rounding adds independent zero-mean noise of at most one
        # bfloat16 ulp (2^-7 relative); a row written k times drifts like sqrt(k) half-ulps.
        # C1 rows are written about 700 times: sqrt(700) * 2^-8 ~ 0.1.
        assert err < 0.1


def test_c3_embedding_error_against_binary64_snapshot():
    """C3's embedding error: bfloat16 tables (binary32 arithmetic, stochastic rounding on
    write-back) trained in SNAPSHOT mode on the first 2^20 samples of C2 (B = 65536, so a
    row is written at most k = 16 times), against the binary64 oracle's SNAPSHOT run:
    ||X - X64||_F / ||X64||_F per table.

    Bound, from the rounding alone: rounding X64 to nearest bfloat16 gives the floor
    e_rne (error variance ulp^2 / 12 per element).  The GPU tables start from the
    round-to-nearest of the initial values and each write adds an independent zero-mean
    stochastic-rounding error of variance p (1 - p) ulp^2 <= ulp^2 / 4, three times the
    nearest-rounding variance, so after k writes the error is at most sqrt(1 + 3k) e_rne;
    binary32 arithmetic adds ~1e-7.  The test allows 1.25 sqrt(1 + 3k) e_rne."""
    import torch
    lh = _lh()
    from test_gpu_parity import _c2
    g, _, _, _ = _c2()
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    count, B, T = 1 << 20, 65536, 200_000_000
    m = oracle.Model(t, d=128, K=5, orders=3, T=T, seed=2)
    m.train(0, count, "snapshot", B)
    tr = trainer_for(g, d=128, K=5, orders=3, dtype="bf16", seed=2, total_samples=T, mode="snapshot", batch=B)
    tr.train_steps(0, count)
    tr.check()
    k = count // B
    for name, tab, ref in (("U", lh.LH_TABLE_U, m.U), ("C", lh.LH_TABLE_C, m.C), ("U1", lh.LH_TABLE_U1, m.U1)):
        err = fro_rel_err(tr.read(tab).cpu().numpy(), ref)
        floor = fro_rel_err(torch.tensor(ref, dtype=torch.float32).to(torch.bfloat16).float().numpy(), ref)
        print(f"C3 embedding error {name}: {err:.3e} (nearest-bf16 floor {floor:.3e}, bound "
              f"{1.25 * (1 + 3 * k) ** 0.5 * floor:.3e})", flush=True)
        assert err <= 1.25 * (1 + 3 * k) ** 0.5 * floor, (name, err, floor)


def test_tune_is_a_dry_run():
    lh = _lh()
    g = rmat_graph(12, 3000, 30_000, seed=5)
    tr = trainer_for(g, d=128, K=5, orders=3, dtype="fp32", seed=6, total_samples=1_000_000)
    before = [tr.read(t).cpu().numpy() for t in (0, 1, 2)]
    tr.tune(probe=200_000)
    after = [tr.read(t).cpu().numpy() for t in (0, 1, 2)]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    cfg = tr.kernel_config()
    assert cfg["lanes_per_sample"] * cfg["units_per_lane"] >= 128


def test_tune_of_bf16_tables_is_a_dry_run():
    """bfloat16 timing runs (step size scaled to zero, hot rows still issuing their packed
    atomics) leave every table bit for bit as it was, and pick a compiled shape that covers
    a row."""
    lh = _lh()
    g = rmat_graph(12, 3000, 30_000, seed=5)
    tr = trainer_for(g, d=128, K=5, orders=3, dtype="bf16", seed=6, total_samples=1_000_000)
    before = [tr.read(t).cpu().numpy() for t in (0, 1, 2)]
    tr.tune(probe=200_000)
    after = [tr.read(t).cpu().numpy() for t in (0, 1, 2)]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    cfg = tr.kernel_config()
    assert cfg["lanes_per_sample"] * cfg["units_per_lane"] == 64
    tr.train_steps(0, 1_000_000)
    tr.check()
    assert np.all(np.isfinite(tr.read(lh.LH_TABLE_U).cpu().numpy()))


# ---------------------------------------------------------------------------
# Batched persistent launch.
# ---------------------------------------------------------------------------
def _small_batch(G=6, dtype="bf16"):
    """The six small graphs of the stored oracle AUCs (or the first G), one Trainer each on
    one shared stream."""
    import torch
    lh = _lh()
    stream = torch.cuda.Stream()
    items = []
    for it in small_batch(G):
        g = it["graph"]
        tr = lh.Trainer(g.n, g.src, g.dst, g.w, d=it["d"], K=5, orders=2, dtype=dtype, seed=it["seed"],
                        graph_id=it["graph_id"], total_samples=it["T"], stream=stream)
        items.append((g, it["held_src"], it["held_dst"], it["neg_dst"], it["T"], it["d"], tr))
    return items


def test_batched_launch_trains_every_sample_once_and_matches_oracle():
    """Six binary32 graphs in one launch: every graph's [0, T) is trained exactly once, and
    each graph's held-out AUCs match the binary64 oracle trained on that graph alone
    within 0.005."""
    lh = _lh()
    gold = json.load(open(os.path.join(GOLDEN, "batch6_oracle_auc.json")))["graphs"]
    items = _small_batch(dtype="fp32")
    bt = lh.BatchTrainer([it[-1] for it in items])
    bt.run()
    assert bt.done() == [it[4] for it in items]
    for gi, (g, hs, hd, neg, T, d, tr) in enumerate(items):
        tr.check()
        uc, uu = _auc_uc_uu(tr, hs, hd, neg)
        ref = gold[gi]
        assert ref["graph_id"] == gi and ref["T"] == T and ref["m_train"] == g.m
        print(f"fp32 graph {gi} (n={g.n}, d={d}): batched uc {uc:.4f} (oracle {ref['auc_uc']:.4f}) "
              f"uu {uu:.4f} (oracle {ref['auc_uu']:.4f})", flush=True)
        assert abs(uc - ref["auc_uc"]) <= 0.005 and abs(uu - ref["auc_uu"]) <= 0.005


def test_batched_bf16_matches_the_oracle_with_bf16_tables():
    """The same six graphs with bfloat16 tables in one launch, against the oracle with
    bfloat16 tables (SEQ, binary64 arithmetic, every write stochastically rounded): on these
    small graphs trained for 20 epochs the rounding itself moves uc by 0.007 to 0.017 from
    the binary64 oracle (the oracle's own bfloat16 runs show it, with no concurrency), and
    makes each run's AUC a random draw with a spread sd_g measured over 8 independent
    rounding streams.  One GPU run is one such draw, so per graph the AUCs must lie within
    0.005 + 3 sd_g sqrt(1 + 1/8) of the oracle's mean (a 0.3 % false-alarm bound for a
    draw of the same distribution), and the mean over the six graphs of the differences
    within 0.005 + 3 sqrt(sum sd_g^2 (1 + 1/8)) / 6."""
    lh = _lh()
    gold = json.load(open(os.path.join(GOLDEN, "batch6_oracle_bf16_auc.json")))
    assert gold["rounding_streams"] == 8
    gold = gold["graphs"]
    b64 = json.load(open(os.path.join(GOLDEN, "batch6_oracle_auc.json")))["graphs"]
    items = _small_batch(dtype="bf16")
    bt = lh.BatchTrainer([it[-1] for it in items])
    bt.run()
    assert bt.done() == [it[4] for it in items]
    diffs = {"uc": [], "uu": []}
    var = {"uc": 0.0, "uu": 0.0}
    for gi, (g, hs, hd, neg, T, d, tr) in enumerate(items):
        tr.check()
        got = dict(zip(("uc", "uu"), _auc_uc_uu(tr, hs, hd, neg)))
        ref = gold[gi]
        assert ref["graph_id"] == gi and ref["T"] == T and ref["m_train"] == g.m
        for k in ("uc", "uu"):
            sd = ref["sd_" + k]
            tol = 0.005 + 3.0 * sd * (1.0 + 1.0 / 8.0) ** 0.5
            print(f"bf16 graph {gi} (n={g.n}, d={d}) {k}: batched {got[k]:.4f}, oracle bf16 tables "
                  f"{ref['auc_' + k]:.4f} (sd {sd:.4f}, bar {tol:.4f}), oracle binary64 {b64[gi]['auc_' + k]:.4f}",
                  flush=True)
            assert abs(got[k] - ref["auc_" + k]) <= tol, (gi, k, got[k], ref["auc_" + k], tol)
            diffs[k].append(got[k] - ref["auc_" + k])
            var[k] += sd * sd * (1.0 + 1.0 / 8.0)
    for k in ("uc", "uu"):
        mean_diff = sum(diffs[k]) / len(diffs[k])
        bar = 0.005 + 3.0 * var[k] ** 0.5 / len(diffs[k])
        print(f"bf16 {k}: mean difference over the graphs {mean_diff:+.4f} (bar {bar:.4f})", flush=True)
        assert abs(mean_diff) <= bar


def test_batched_launch_on_the_callers_stream():
    """A captured batch replayed on another stream waits for the work queued before it on
    the trainers' stream (here: the initial values) and the trainers' stream waits for it:
    reading the tables right after gives the trained tables, equal in count of samples and
    in AUC to a replay on the trainers' own stream."""
    import torch
    lh = _lh()
    gold = json.load(open(os.path.join(GOLDEN, "batch6_oracle_auc.json")))["graphs"]
    items = _small_batch(G=3, dtype="fp32")
    bt = lh.BatchTrainer([it[-1] for it in items])
    bt.capture()
    other = torch.cuda.Stream()
    for it in items:
        it[-1].init_embeddings()
    bt.launch(other)
    assert bt.done() == [it[4] for it in items]
    for gi, (g, hs, hd, neg, T, d, tr) in enumerate(items):
        uc, uu = _auc_uc_uu(tr, hs, hd, neg)
        print(f"graph {gi} on another stream: uc {uc:.4f} (oracle {gold[gi]['auc_uc']:.4f})", flush=True)
        assert abs(uc - gold[gi]["auc_uc"]) <= 0.005 and abs(uu - gold[gi]["auc_uu"]) <= 0.005


def test_batched_graph_capture_replays():
    lh = _lh()
    items = _small_batch(G=4)
    bt = lh.BatchTrainer([it[-1] for it in items])
    bt.capture()
    for rep in range(3):
        bt.launch()
        ms = bt.last_ms()
        assert bt.done() == [it[4] for it in items], rep
        assert ms > 0
        for it in items:
            x = it[-1].read(lh.LH_TABLE_U).cpu().numpy()
            assert np.all(np.isfinite(x))


def test_batched_tuner_is_a_dry_run():
    lh = _lh()
    items = _small_batch(G=3, dtype="fp32")
    trs = [it[-1] for it in items]
    before = [t.read(lh.LH_TABLE_C).cpu().numpy() for t in trs]
    bt = lh.BatchTrainer(trs)
    bt.tune()
    after = [t.read(lh.LH_TABLE_C).cpu().numpy() for t in trs]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    bt.run()
    assert bt.done() == [it[4] for it in items]


def test_batched_tuner_of_bf16_is_a_dry_run():
    lh = _lh()
    items = _small_batch(G=3, dtype="bf16")
    trs = [it[-1] for it in items]
    before = [t.read(lh.LH_TABLE_C).cpu().numpy() for t in trs]
    bt = lh.BatchTrainer(trs)
    bt.tune()
    after = [t.read(lh.LH_TABLE_C).cpu().numpy() for t in trs]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    bt.run()
    assert bt.done() == [it[4] for it in items]


# ---------------------------------------------------------------------------
# Kernel configuration and the bfloat16 shadow's capacity.
# ---------------------------------------------------------------------------
def test_set_kernel_config_checks_the_shape():
    lh = _lh()
    g = rmat_graph(12, 3000, 30_000, seed=5)
    tr = trainer_for(g, d=128, K=5, orders=2, dtype="bf16", seed=6, total_samples=1_000_000)
    tr.set_kernel_config(32, 2, 4)
    assert tr.kernel_config() == {"lanes_per_sample": 32, "units_per_lane": 2, "blocks_per_cu": 4}
    for bad in ((16, 2, 4),   # 32 units < the 64 units of a bf16 row of 128
                (8, 1, 4),    # not a compiled shape
                (64, 1, 0), (64, 1, 65)):
        with pytest.raises(lh.LhError) as e:
            tr.set_kernel_config(*bad)
        assert e.value.status == 1
    assert tr.kernel_config() == {"lanes_per_sample": 32, "units_per_lane": 2, "blocks_per_cu": 4}
    tr.train_steps(0, 100_000)
    tr.check()
    assert np.all(np.isfinite(tr.read(lh.LH_TABLE_U).cpu().numpy()))


def test_bf16_shadow_capacity_with_imported_tables():
    """(bfloat16 with the binary32 shadow of the hot rows.)  Imported alias tables carry no
    degrees, so every node asks for a shadow slot; with
    more nodes than the shadow holds (n = 150,000 > 131,072 slots) the first 131,072 get
    one and the rest take the table path.  Training must stay sound: finite tables and
    held-out AUC close to the same run on tables built (with degrees) on the device."""
    lh = _lh()
    g0 = rmat_graph(18, 150_000, 1_500_000, seed=41)
    from synth.graphs import auc_negatives, holdout_split
    g, hs, hd = holdout_split(g0, seed=42)
    neg = auc_negatives(g0.n, g0.src, g0.dst, hs, seed=43)
    T = 10 * g.m
    built = trainer_for(g, d=64, K=5, orders=2, dtype="bf16", seed=7, total_samples=T, hot_shadow=True)
    imp = trainer_for(g, d=64, K=5, orders=2, dtype="bf16", seed=7, total_samples=T, build=False, hot_shadow=True)
    for which in (lh.LH_ALIAS_EDGE, lh.LH_ALIAS_NEG):
        thr, al = built.export_alias(which)
        imp.import_alias(which, thr, al)
    imp.check()
    results = []
    for tr in (built, imp):
        tr.train_steps(0, T)
        tr.check()
        for t in (lh.LH_TABLE_U, lh.LH_TABLE_C):
            assert np.all(np.isfinite(tr.read(t).cpu().numpy()))
        results.append(_auc_uc_uu(tr, hs, hd, neg))
    print(f"n={g.n}: built uc {results[0][0]:.4f} uu {results[0][1]:.4f}; imported uc {results[1][0]:.4f} "
          f"uu {results[1][1]:.4f}", flush=True)
    assert abs(results[0][0] - results[1][0]) <= 0.01 and abs(results[0][1] - results[1][1]) <= 0.01


def test_bf16_shape_follows_the_hot_share():
    """Without a pinned shape, a bfloat16 handle runs two samples per wavefront when few
    row touches fall on hot rows (uniform endpoints, 2^20 nodes: no row reaches the hot
    rate) and one sample per wavefront where hub rows take most touches (the R-MAT mid
    graph: about two thirds of the touches go to hot rows); a pinned shape survives a
    rebuild of the alias tables."""
    import torch
    lh = _lh()
    from synth.graphs import mid_graph, uniform_graph_gpu
    src, dst, w = uniform_graph_gpu(1 << 20, 1 << 24, seed=9)
    torch.cuda.synchronize()
    uni = lh.Trainer(1 << 20, src, dst, w, d=128, K=5, orders=2, dtype="bf16", seed=9, total_samples=10_000_000)
    assert uni.kernel_config() == {"lanes_per_sample": 32, "units_per_lane": 2, "blocks_per_cu": 16}
    uni.train_steps(0, 10_000_000)
    uni.check()
    assert np.all(np.isfinite(uni.read(lh.LH_TABLE_C).cpu().numpy()))
    uni.set_kernel_config(64, 1, 16)
    uni.build_alias()
    assert uni.kernel_config() == {"lanes_per_sample": 64, "units_per_lane": 1, "blocks_per_cu": 16}
    uni.close()
    del src, dst, w
    g = mid_graph()["graph"]
    hub = trainer_for(g, d=128, K=5, orders=2, dtype="bf16", seed=7, total_samples=10 * g.m)
    assert hub.kernel_config() == {"lanes_per_sample": 64, "units_per_lane": 1, "blocks_per_cu": 16}


@pytest.mark.parametrize("dtype,d,shape", [("fp32", 64, None), ("bf16", 64, None), ("fp32", 128, (64, 2, 4))])
def test_hot_and_cold_writes_agree_bitwise_without_concurrency(dtype, d, shape):
    """One sample per launch, so no write overlaps another: a run where every row takes the
    atomic (hot) path must leave the tables bit-identical to a run where every row takes the
    store (cold) path.  binary32: old + inc rounded once either way.  bfloat16: the packed
    atomic adds SR(old + inc) - old, drawn with the cold store's random bits; that
    difference is exact (Sterbenz) while old and SR(old + inc) are within a factor of two,
    so the tables start with every |value| in [2^-6, 2^-5) and the step stays far below
    that (the general case is bounded in tests/test_bf16_rounding.py).  The binary32 case at
    the C2 tile shape (one sample per wavefront) writes cold rows with the streaming buffer
    stores."""
    lh = _lh()
    g = rmat_graph(12, 3000, 30_000, seed=11)
    rng = np.random.default_rng(13)
    start = [(rng.choice([-1.0, 1.0], (g.n, d)) * (1.0 + rng.integers(0, 128, (g.n, d)) / 128.0) * 2.0 ** -6)
             .astype(np.float32) for _ in range(3)]
    out = []
    for hot_rate in (0.0, 1e31):  # <= 0: every row hot; >= 1e30: none
        tr = trainer_for(g, d=d, K=5, orders=3, dtype=dtype, seed=12, total_samples=10_000, hot_rate=hot_rate)
        if shape is not None:
            tr.set_kernel_config(*shape)
        for t in (lh.LH_TABLE_U, lh.LH_TABLE_C, lh.LH_TABLE_U1):
            tr.write(t, start[t])
        for s in range(300):
            tr.train_steps(s, 1)
        tr.check()
        out.append([tr.read(t).cpu().numpy() for t in (lh.LH_TABLE_U, lh.LH_TABLE_C, lh.LH_TABLE_U1)])
        tr.close()
    for a, b, a0 in zip(*out, start):
        assert not np.array_equal(a, a0)  # the samples did change the tables
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
