"""The seeded input generators: determinism and the stated workload shapes."""
import numpy as np

from synth import CONFIGS, auc_negatives, batch_graph_specs, config_graph, holdout_split, rmat_graph


def test_rmat_is_deterministic_and_clean():
    a = rmat_graph(12, 3000, 20_000, seed=5, directed=True, weights="lognormal")
    b = rmat_graph(12, 3000, 20_000, seed=5, directed=True, weights="lognormal")
    c = rmat_graph(12, 3000, 20_000, seed=6, directed=True, weights="lognormal")
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst) and np.array_equal(a.w, b.w)
    assert not np.array_equal(a.src, c.src)
    assert a.m == 20_000 and a.src.max() < 3000 and np.all(a.src != a.dst)
    keys = a.src.astype(np.int64) * a.n + a.dst
    assert np.unique(keys).size == a.m
    assert a.w.dtype == np.float32 and np.all(a.w > 0)


def test_c1_shape(c1_graph):
    g = c1_graph
    cfg = CONFIGS["C1"]
    assert g.n == cfg["n"] and g.m == 2 * cfg["m_unique"]
    assert np.array_equal(g.src[0::2], g.dst[1::2]) and np.array_equal(g.dst[0::2], g.src[1::2])
    assert np.all(g.w == 1.0) and np.all(g.src != g.dst)
    lo = np.minimum(g.src[0::2], g.dst[0::2]).astype(np.int64)
    hi = np.maximum(g.src[0::2], g.dst[0::2]).astype(np.int64)
    assert np.unique(lo * g.n + hi).size == cfg["m_unique"]


def test_holdout_and_negatives():
    g = rmat_graph(10, 1000, 5000, seed=9, directed=True)
    tr, hs, hd = holdout_split(g, seed=3)
    assert hs.size == 50 and tr.m == 4950
    neg = auc_negatives(g.n, g.src, g.dst, hs, seed=4)
    keys = set((g.src.astype(np.int64) * g.n + g.dst).tolist())
    assert all(int(u) * g.n + int(v) not in keys for u, v in zip(hs, neg))
    assert np.all(neg != hs)


def test_c1_auc_variant():
    tr, hs, hd, neg = config_graph("C1", holdout=True)
    assert hs.size == 2000 and tr.m == 198_000


def test_batch_specs():
    specs = batch_graph_specs()
    assert len(specs) == 64
    assert all(1000 <= s["n"] <= 2_000_000 and s["d"] in (64, 128) for s in specs)
    assert all(8 <= s["m"] / s["n"] <= 32.01 for s in specs)
    assert specs == batch_graph_specs()


def test_small_batch_matches_stored_oracle_aucs():
    """The stored batch oracle AUCs were computed on exactly these graphs."""
    import json
    import os
    from synth import small_batch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch6_oracle_auc.json")))
    for it, ref in zip(small_batch(6), gold["graphs"]):
        assert (it["graph"].n, it["graph"].m, it["held_src"].size, it["d"], it["T"], it["seed"]) == \
            (ref["n"], ref["m_train"], ref["held_out"], ref["d"], ref["T"], ref["seed"])


def test_mid_graph_matches_stored_oracle_aucs():
    import json
    import os
    from synth import mid_graph
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mid_oracle_auc.json")))
    it = mid_graph()
    assert (it["graph"].n, it["graph"].m, it["held_src"].size, it["T"], it["seed"]) == \
        (gold["n"], gold["m_train"], gold["held_out"], gold["T"], gold["seed"])
