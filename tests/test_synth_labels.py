"""The labelled stand-in graphs (stochastic block model) and the node-classification
score (Sec. V-A: one-vs-rest logistic regression on 10 % of the labels, Micro/Macro-F1)."""
import numpy as np

from synth.labels import SBM, node_classification_f1, sbm_graph, sbm_workload


def test_sbm_is_deterministic_and_clean():
    g, lab = sbm_graph(3000, 5, 12.0, 0.6, seed=4)
    g2, lab2 = sbm_graph(3000, 5, 12.0, 0.6, seed=4)
    assert np.array_equal(g.src, g2.src) and np.array_equal(lab, lab2)
    assert g.m == 2 * 18_000 and lab.size == 3000 and set(np.unique(lab)) == set(range(5))
    assert np.array_equal(g.src[0::2], g.dst[1::2]) and np.array_equal(g.dst[0::2], g.src[1::2])
    assert np.all(g.src != g.dst) and np.all(g.w == 1.0)
    a = np.minimum(g.src[0::2], g.dst[0::2]).astype(np.int64)
    b = np.maximum(g.src[0::2], g.dst[0::2]).astype(np.int64)
    assert np.unique(a * g.n + b).size == 18_000


def test_sbm_in_class_share_matches_the_recipe():
    g, lab = sbm_graph(20_000, 10, 20.0, 0.5, seed=9)
    share = np.mean(lab[g.src] == lab[g.dst])
    sizes = np.bincount(lab) / lab.size
    # a draw is inside its class with probability p_in + (1 - p_in) * P(uniform partner shares the class)
    want = 0.5 + 0.5 * np.sum(sizes * sizes)
    assert abs(share - want) < 0.01, (share, want)


def test_f1_of_separable_and_of_random_features():
    rng = np.random.default_rng(0)
    lab = rng.integers(0, 6, size=5000).astype(np.int32)
    onehot = np.eye(6)[lab] + 0.01 * rng.normal(size=(5000, 6))
    mi, ma = node_classification_f1(onehot, lab, seed=1)
    assert mi > 0.99 and ma > 0.99
    mi, ma = node_classification_f1(rng.normal(size=(5000, 16)), lab, seed=1)
    assert mi < 0.25 and ma < 0.25  # six classes: chance is about 1/6


def test_sbm_workload_shape():
    g, lab, c = sbm_workload()
    assert g.n == SBM["n"] and g.m == 2 * SBM["n"] * SBM["mean_degree"] / 2 and c["T"] == SBM["epochs"] * g.m
