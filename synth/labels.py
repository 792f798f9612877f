"""Labelled synthetic graphs and the node-classification score of embeddings.

The paper measures embedding quality by multi-class node classification (Sec. V-A): a
one-vs-rest logistic regression trained on 10 % of the nodes' labels, scored by Micro-
and Macro-F1 on the rest.  Its labelled datasets (Table II) are not available here; a
stochastic block model with planted classes stands in for them.

Nothing here is the embedding method's arithmetic: the generator only produces arrays,
and the score uses scikit-learn's logistic regression and F1 on embeddings given to it.
"""
from __future__ import annotations

import numpy as np

from .graphs import Graph


def sbm_graph(n: int, classes: int, mean_degree: float, p_in: float, seed: int):
    """Undirected stochastic block model with planted classes.

    Class sizes: a seeded multinomial split of n with class weights uniform on [0.5, 1.5].
    Edges: n * mean_degree / 2 unique undirected edges; each draw picks u uniformly, then
    with probability p_in a partner uniform in u's class, else one uniform over all nodes;
    self-loops and repeats are dropped (first occurrence kept) and drawing continues to
    the exact count.  Every edge is stored as two arcs, (u, v) then (v, u), weight 1.
    Returns (graph, labels int32[n])."""
    rng = np.random.default_rng(seed)
    wts = rng.uniform(0.5, 1.5, size=classes)
    sizes = rng.multinomial(n - classes, wts / wts.sum()) + 1
    labels = rng.permutation(np.repeat(np.arange(classes, dtype=np.int32), sizes))
    members = [np.flatnonzero(labels == c) for c in range(classes)]
    m_unique = int(round(n * mean_degree / 2))
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m_unique:
        cnt = int((m_unique - keys.size) * 1.2) + 1024
        u = rng.integers(0, n, size=cnt)
        inside = rng.random(cnt) < p_in
        v = rng.integers(0, n, size=cnt)
        lu = labels[u]
        r = rng.random(cnt)
        for c in range(classes):
            sel = inside & (lu == c)
            v[sel] = members[c][(r[sel] * members[c].size).astype(np.int64)]
        ok = u != v
        a, b = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
        allk = np.concatenate([keys, a.astype(np.int64) * n + b])
        _, first = np.unique(allk, return_index=True)
        keys = allk[np.sort(first)]
    keys = keys[:m_unique]
    a, b = (keys // n).astype(np.int32), (keys % n).astype(np.int32)
    src = np.empty(2 * m_unique, np.int32)
    dst = np.empty(2 * m_unique, np.int32)
    src[0::2], dst[0::2] = a, b
    src[1::2], dst[1::2] = b, a
    g = Graph(n=n, src=src, dst=dst, w=np.ones(2 * m_unique, np.float32), directed=False,
              meta=dict(kind="sbm", classes=classes, mean_degree=mean_degree, p_in=p_in, seed=seed))
    return g, labels


# The labelled workload: 20,000 nodes in 10 classes, mean degree 20, 40 % of the edge draws
# inside a class (Micro-F1 about 0.83 after training: with half the draws inside, F1
# saturates at 0.985, and with 30 % it is 0.36 with a seed-to-seed spread of 0.01);
# d = 128, K = 5, second order, 100 epochs (T = 100 m: with 25 epochs at eta0 = 0.025
# the vertex rows are still all aligned with one direction and carry no class signal).
SBM = dict(n=20_000, classes=10, mean_degree=20.0, p_in=0.4, seed=61, d=128, K=5, orders=2, epochs=100,
           train_seed=62, eta0=0.025, split_seed=63)


def sbm_workload():
    c = SBM
    g, labels = sbm_graph(c["n"], c["classes"], c["mean_degree"], c["p_in"], c["seed"])
    return g, labels, dict(c, T=c["epochs"] * g.m)


def node_classification_f1(X, labels, seed: int, train_frac: float = 0.1):
    """Micro- and Macro-F1 of a one-vs-rest logistic regression (scikit-learn, C = 1,
    L-BFGS) on the L2-normalised rows of X, trained on a seeded random train_frac of the
    nodes and scored on the rest."""
    from sklearn.linear_model import LogisticRegression
    from sklearn.metrics import f1_score
    from sklearn.multiclass import OneVsRestClassifier
    X = np.asarray(X, dtype=np.float64)
    norms = np.linalg.norm(X, axis=1, keepdims=True)
    X = X / np.where(norms > 0, norms, 1.0)
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    idx = rng.permutation(n)
    k = int(round(train_frac * n))
    tr, te = idx[:k], idx[k:]
    clf = OneVsRestClassifier(LogisticRegression(C=1.0, max_iter=2000))
    clf.fit(X[tr], labels[tr])
    pred = clf.predict(X[te])
    return (float(f1_score(labels[te], pred, average="micro")),
            float(f1_score(labels[te], pred, average="macro")))
