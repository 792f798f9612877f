"""Pins of the oracle's random-walk pair source (Sec. IV-B: Algorithm 2, RandomWalk, and
Algorithm 3, GeneratePairs, on one process, where every vertex is local), against facts
that do not come from the oracle itself:

* the walk graph's rows equal an independent construction (a stable sort of the forward
  and backward entries by tail);
* every row's alias table encodes that row's neighbour weights (exact implied
  probabilities against w / W within the construction's error bound), hub rows spanning
  several scan chunks included;
* walks start with an arc and continue along edges of positive weight, visiting exactly L
  vertices;
* the roots follow the weight-normalised edge distribution, and each step the weights of
  the current vertex's neighbourhood (chi-square);
* the distribution of whole walk prefixes (w0, w1, w2, w3) on a tiny graph equals the
  brute-force product of the root and transition probabilities;
* the pairs of a walk batch are every (walk, pair) once, a window of 2 giving the
  consecutive pairs of each walk;
* training one walk sample applies the per-sample rule (pinned by finite differences in
  the edge-sampling pins) to that sample's pair and negatives, and SNAPSHOT with B = 1 is
  SEQ.

Planted mistakes in copies of the oracle (drawing from the previous vertex's
neighbourhood, a reversed root, neighbours drawn without their weights, a walk one vertex
short, rows out of entry order, a window one too wide) must fail.
"""
import math
import os
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from synth.graphs import Graph

from test_oracle_pins import alias_error_bound, implied_probabilities, implied_probabilities_f64, EPS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")


def _graph(seed, n, m, zero_frac=0.1):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m)
    off = rng.integers(1, n, size=m)
    dst = (src + off) % n
    w = rng.lognormal(0, 1.0, size=m) * (rng.random(m) >= zero_frac)
    w[0] = max(w[0], 0.5)
    return Graph(n=n, src=src.astype(np.int32), dst=dst.astype(np.int32), w=w.astype(np.float32))


def _hub_graph():
    """A random graph plus a hub joined to 3000 vertices (a row of several scan chunks)."""
    g = _graph(7, 4000, 6000)
    rng = np.random.default_rng(8)
    leaves = rng.permutation(np.arange(1, 4000))[:3000]
    src = np.concatenate([g.src, np.zeros(1500, np.int32), leaves[1500:].astype(np.int32)])
    dst = np.concatenate([g.dst, leaves[:1500].astype(np.int32), np.zeros(1500, np.int32)])
    w = np.concatenate([g.w, rng.lognormal(0, 1.5, 3000).astype(np.float32)])
    return Graph(n=4000, src=src, dst=dst, w=w)


def _walker(g, L=100, W=2, Bw=64):
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    return t, oracle.WalkGraph(t, L=L, W=W, Bw=Bw)


# ---------------------------------------------------------------------------
# The walk graph and its per-row tables.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["random", "hub"])
def test_rows_equal_a_stable_sort_of_both_directions(which):
    g = _graph(1, 300, 2000) if which == "random" else _hub_graph()
    _, wg = _walker(g)
    tails = np.concatenate([g.src, g.dst]).astype(np.int64)
    heads = np.concatenate([g.dst, g.src])
    wts = np.concatenate([g.w, g.w]).astype(np.float64)
    order = np.argsort(tails, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(tails, minlength=g.n))])
    assert np.array_equal(wg.off, off)
    assert np.array_equal(wg.nbr, heads[order])
    assert np.array_equal(wg.wt, wts[order])


@pytest.mark.parametrize("which", ["random", "hub"])
def test_row_tables_encode_the_neighbour_weights(which):
    g = _graph(2, 300, 2000) if which == "random" else _hub_graph()
    _, wg = _walker(g)
    checked = 0
    for x in range(g.n):
        lo, hi = int(wg.off[x]), int(wg.off[x + 1])
        if hi == lo:
            continue
        w = wg.wt[lo:hi]
        thr, al = wg.thr[lo:hi], wg.alias[lo:hi]
        assert np.all((al >= 0) & (al < hi - lo))
        if w.sum() == 0:
            assert np.all(thr == np.uint64(2**64 - 1)) and np.array_equal(al, np.arange(hi - lo))
            continue
        if hi - lo <= 40:
            P = implied_probabilities(thr, al)
            W = math.fsum(w)
            bound = alias_error_bound(w, thr, al)
            for i in range(hi - lo):
                assert abs(float(P[i] - Fraction(w[i]) / Fraction(W))) <= bound[i], (x, i)
        else:
            P = implied_probabilities_f64(thr, al)
            p = w / math.fsum(w)
            bound = alias_error_bound(w, thr, al) + 4 * EPS * p + 2.0**-60 / (hi - lo)
            assert np.all(np.abs(P - p) <= bound), x
        checked += 1
    assert checked > 100
    if which == "hub":
        assert wg.off[1] - wg.off[0] > 2048


# ---------------------------------------------------------------------------
# Walks.
# ---------------------------------------------------------------------------
def _entry_weights(g):
    """Total weight of the entries x -> y of the walk graph, as a dict."""
    tot = {}
    for a, b, w in zip(np.concatenate([g.src, g.dst]), np.concatenate([g.dst, g.src]), np.concatenate([g.w, g.w])):
        tot[(int(a), int(b))] = tot.get((int(a), int(b)), 0.0) + float(w)
    return tot


def test_walks_start_with_an_arc_follow_edges_and_visit_L_vertices():
    g = _graph(3, 200, 800)
    _, wg = _walker(g, L=30)
    walks = wg.walks(seed=5, graph_id=1, k0=10**12, nwalks=1500)
    assert walks.shape == (1500, 30)
    arcs = {}
    for a, b, w in zip(g.src, g.dst, g.w):
        arcs[(int(a), int(b))] = arcs.get((int(a), int(b)), 0.0) + float(w)
    ent = _entry_weights(g)
    for row in walks:
        assert arcs.get((int(row[0]), int(row[1])), 0.0) > 0.0
        for t in range(1, 29):
            assert ent.get((int(row[t]), int(row[t + 1])), 0.0) > 0.0, (t, row[t], row[t + 1])


def _chisq_rows(counts, probs, min_expected=5.0):
    """Goodness of fit of per-row categorical counts: cells with expectation below
    min_expected are pooled per row; returns the p-value of the summed statistic."""
    stat, df = 0.0, 0
    for c, p in zip(counts, probs):
        n = c.sum()
        if n == 0:
            continue
        e = p * n
        big = e >= min_expected
        cc = np.concatenate([c[big], [c[~big].sum()]]) if (~big).any() else c[big]
        ee = np.concatenate([e[big], [e[~big].sum()]]) if (~big).any() else e[big]
        keep = ee > 0
        cc, ee = cc[keep], ee[keep]
        if cc.size < 2:
            continue
        stat += float(((cc - ee) ** 2 / ee).sum())
        df += cc.size - 1
    return stats.chi2.sf(stat, df)


def test_roots_follow_the_edge_distribution():
    g = _graph(4, 100, 400)
    _, wg = _walker(g, L=2, W=2, Bw=1000)
    u, v = wg.pairs(seed=9, graph_id=0, first=0, count=400_000)
    key = u.astype(np.int64) * g.n + v
    akey = g.src.astype(np.int64) * g.n + g.dst
    uk, inv = np.unique(akey, return_inverse=True)
    wsum = np.bincount(inv, weights=g.w.astype(np.float64), minlength=uk.size)
    pos = np.searchsorted(uk, key)
    assert np.all(uk[np.minimum(pos, uk.size - 1)] == key)
    counts = np.bincount(pos, minlength=uk.size).astype(np.float64)
    assert _chisq_rows([counts], [wsum / wsum.sum()]) > 1e-3


def test_steps_follow_the_neighbour_weights():
    g = _graph(5, 60, 300)
    _, wg = _walker(g, L=40)
    walks = wg.walks(seed=3, graph_id=0, k0=0, nwalks=20_000)
    cur = walks[:, 1:-1].ravel().astype(np.int64)
    nxt = walks[:, 2:].ravel().astype(np.int64)
    counts = np.zeros((g.n, g.n))
    np.add.at(counts, (cur, nxt), 1.0)
    P = np.zeros((g.n, g.n))
    for (a, b), w in _entry_weights(g).items():
        P[a, b] += w
    rows = P.sum(axis=1) > 0
    P[rows] /= P[rows].sum(axis=1, keepdims=True)
    assert counts[~rows].sum() == 0
    assert _chisq_rows(counts[rows], P[rows]) > 1e-3


def test_walk_prefixes_match_the_brute_force_distribution():
    """(w0, w1, w2, w3) of walks on a 5-vertex graph: probability = P(root arc (w0, w1))
    p(w2 | w1) p(w3 | w2), enumerated exactly."""
    src = np.array([0, 1, 2, 3, 0, 4, 2, 1], np.int32)
    dst = np.array([1, 2, 3, 0, 2, 1, 4, 3], np.int32)
    w = np.array([1.0, 2.5, 0.7, 3.0, 1.8, 0.4, 2.2, 1.1], np.float32)
    g = Graph(n=5, src=src, dst=dst, w=w)
    _, wg = _walker(g, L=4, Bw=1)
    walks = wg.walks(seed=11, graph_id=0, k0=0, nwalks=300_000)
    ent = _entry_weights(g)
    out = {}
    for a, b in ent:
        out.setdefault(a, []).append(b)
    strength = {x: sum(ent[(x, y)] for y in out[x]) for x in out}
    W = math.fsum(float(x) for x in w)
    probs = {}
    for a, b, wa in zip(src, dst, w):
        for c in out[int(b)]:
            for d in out[c]:
                p = float(wa) / W * ent[(int(b), c)] / strength[int(b)] * ent[(c, d)] / strength[c]
                key = (int(a), int(b), c, d)
                probs[key] = probs.get(key, 0.0) + p
    keys = sorted(probs)
    index = {k: i for i, k in enumerate(keys)}
    counts = np.zeros(len(keys))
    for row in walks:
        k = tuple(int(x) for x in row)
        assert k in index, k
        counts[index[k]] += 1
    p = np.array([probs[k] for k in keys])
    assert abs(p.sum() - 1.0) < 1e-12
    assert _chisq_rows([counts], [p]) > 1e-3


# ---------------------------------------------------------------------------
# Pairs and their sample order.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,W,Bw", [(7, 2, 5), (7, 3, 5), (100, 2, 3)])
def test_a_batch_holds_every_pair_of_every_walk_once(L, W, Bw):
    g = _graph(6, 80, 300)
    _, wg = _walker(g, L=L, W=W, Bw=Bw)
    P = sum(L - dl for dl in range(1, W))
    assert wg.pairs_per_walk == P
    for b in (0, 3):
        u, v = wg.pairs(seed=2, graph_id=0, first=b * Bw * P, count=Bw * P)
        walks = wg.walks(seed=2, graph_id=0, k0=b * Bw, nwalks=Bw)
        want = sorted((j, int(walks[j, i]), int(walks[j, i + dl])) for j in range(Bw) for dl in range(1, W)
                      for i in range(L - dl))
        # sample b Bw P + p Bw + j belongs to walk j of the batch
        got = sorted((idx % Bw, int(u[idx]), int(v[idx])) for idx in range(Bw * P))
        assert got == want
        # consecutive samples come from different walks (Bw > 1)
        if Bw > 1:
            j = np.arange(Bw * P) % Bw
            assert np.all(j[1:] != j[:-1])
    if W == 2:
        u, v = wg.pairs(seed=2, graph_id=0, first=0, count=Bw * P)
        walks = wg.walks(seed=2, graph_id=0, k0=0, nwalks=Bw)
        for j in range(Bw):
            assert np.array_equal(u[j::Bw], walks[j, :-1]) and np.array_equal(v[j::Bw], walks[j, 1:])


def test_pairs_of_any_range_are_the_batch_pairs():
    g = _graph(6, 80, 300)
    _, wg = _walker(g, L=9, W=3, Bw=4)
    per = 4 * wg.pairs_per_walk
    u, v = wg.pairs(seed=1, graph_id=2, first=2**33, count=3 * per)
    for off in (0, 7, per - 3, per + 5):
        uu, vv = wg.pairs(seed=1, graph_id=2, first=2**33 + off, count=11)
        assert np.array_equal(uu, u[off:off + 11]) and np.array_equal(vv, v[off:off + 11])


# ---------------------------------------------------------------------------
# Training with walk pairs.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("s", [0, 1, 250, 999])
@pytest.mark.parametrize("orders", [2, 1, 3])
def test_one_walk_sample_applies_the_per_sample_rule(s, orders):
    g = _graph(9, 50, 200, zero_frac=0.0)
    t, wg = _walker(g, L=12, W=2, Bw=8)
    K, T, eta0 = 3, 1000, 0.4
    m = oracle.Model(t, d=8, K=K, orders=orders, T=T, seed=4, eta0=eta0, lam=0.01, alpha=0.7)
    rng = np.random.default_rng(s)
    for X in (m.U, m.C, m.U1):
        if X is not None:
            X[:] = rng.normal(0, 0.3, size=X.shape)
    ref = {k: (None if X is None else X.copy()) for k, X in (("U", m.U), ("C", m.C), ("U1", m.U1))}
    m.train(s, 1, "seq", walks=wg)
    u, v = wg.pairs(seed=4, graph_id=0, first=s, count=1)
    neg = oracle.sample_negatives(g.n, t.nthr, t.nalias, seed=4, graph_id=0, K=K, first=s, count=1)[0]
    ids = np.concatenate([[v[0]], neg]).astype(np.int32)
    eta = eta0 * (1.0 - s / T)
    if orders & 2:
        oracle.apply_tuple(ref["U"], ref["C"], int(u[0]), ids, eta, 0.01, 0.7)
    if orders & 1:
        oracle.apply_tuple(ref["U1"], ref["U1"], int(u[0]), ids, eta, 0.01, 0.7)
    for k, X in (("U", m.U), ("C", m.C), ("U1", m.U1)):
        if X is not None:
            assert np.array_equal(X, ref[k]), k


def _bf16_neighbours(x):
    f = np.float32(x)
    b = f.view(np.uint32)
    lo = np.uint32(b & np.uint32(0xFFFF0000)).view(np.float32)
    if np.uint32(b & np.uint32(0xFFFF)) == 0:
        return float(lo), float(lo)
    hi = np.uint32((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32)
    return float(lo), float(hi)


@pytest.mark.parametrize("s", [0, 77, 500])
def test_one_bf16_walk_sample_lands_next_to_the_binary64_step(s):
    """bfloat16 storage with walk pairs: one sample writes exactly the rows of its walk
    pair and negatives, each element once written on a bfloat16 neighbour of the binary64
    step from the same tables; a zero step leaves the tables as they were."""
    g = _graph(12, 40, 160, zero_frac=0.0)
    t, wg = _walker(g, L=8, W=2, Bw=4)
    K = 2
    a = oracle.Model(t, d=16, K=K, orders=2, T=1000, seed=3, eta0=0.5, storage="bf16")
    b = oracle.Model(t, d=16, K=K, orders=2, T=1000, seed=3, eta0=0.5)
    rng = np.random.default_rng(s)
    for X, Y in ((a.U, b.U), (a.C, b.C)):
        X[:] = oracle.bf16_rne(rng.normal(0, 0.3, size=X.shape))
        Y[:] = X
    before = (a.U.copy(), a.C.copy())
    a.train(s, 1, "seq", walks=wg)
    b.train(s, 1, "seq", walks=wg)
    u, v = wg.pairs(seed=3, graph_id=0, first=s, count=1)
    neg = oracle.sample_negatives(g.n, t.nthr, t.nalias, seed=3, graph_id=0, K=K, first=s, count=1)[0]
    ids = [int(v[0])] + [int(x) for x in neg]
    for X, Y, X0, rows in ((a.U, b.U, before[0], [int(u[0])]), (a.C, b.C, before[1], ids)):
        untouched = np.setdiff1d(np.arange(X.shape[0]), rows)
        assert np.array_equal(X[untouched], X0[untouched])
        for r in set(rows):
            if rows.count(r) != 1:
                continue
            for c in range(X.shape[1]):
                assert X[r, c] in _bf16_neighbours(Y[r, c]), (r, c)
    z = oracle.Model(t, d=16, K=K, orders=2, T=1000, seed=3, eta0=0.0, storage="bf16")
    z0 = (z.U.copy(), z.C.copy())
    z.train(0, 300, "seq", walks=wg)
    assert np.array_equal(z.U, z0[0]) and np.array_equal(z.C, z0[1])


def test_walk_snapshot_with_batch_one_is_seq():
    g = _graph(10, 120, 600, zero_frac=0.0)
    t, wg = _walker(g, L=10, W=2, Bw=16)
    a = oracle.Model(t, d=16, K=2, orders=3, T=5000, seed=6, eta0=0.2)
    b = oracle.Model(t, d=16, K=2, orders=3, T=5000, seed=6, eta0=0.2)
    a.train(37, 3000, "seq", walks=wg)
    b.train(37, 3000, "snapshot", 1, walks=wg)
    for x, y in ((a.U, b.U), (a.C, b.C), (a.U1, b.U1)):
        assert np.max(np.abs(x - y)) <= 1e-14


def test_walk_snapshot_needs_batches_inside_walk_batches():
    g = _graph(10, 120, 600)
    t, wg = _walker(g, L=10, W=2, Bw=16)  # 144 samples per walk batch
    m = oracle.Model(t, d=8, K=1, orders=2, T=5000, seed=6)
    m.train(0, 288, "snapshot", 48, walks=wg)
    with pytest.raises(ValueError):
        m.train(0, 100, "snapshot", 100, walks=wg)


# ---------------------------------------------------------------------------
# Planted mistakes.
# ---------------------------------------------------------------------------
MUTATIONS = {
    "previous vertex's neighbourhood": (
        "int64_t lo = wk->off[vert[t]], len = wk->off[vert[t] + 1] - lo;",
        "int64_t lo = wk->off[vert[t - 1]], len = wk->off[vert[t - 1] + 1] - lo;"),
    "reversed root": ("    vert[0] = wk->src[a];\n    vert[1] = wk->dst[a];",
                      "    vert[0] = wk->dst[a];\n    vert[1] = wk->src[a];"),
    "unweighted neighbours": (
        "int64_t item = draw(wk->wthr + lo, wk->walias + lo, len, x[0], x[1]);",
        "int64_t item = (int64_t)(((u128)x[0] * (uint64_t)len) >> 64);"),
    "one vertex short": ("for (int t = 1; t + 1 < wk->L; t++) {", "for (int t = 1; t + 2 < wk->L; t++) {"),
    "rows out of entry order": ("for (int64_t e = 0; e < 2 * m; e++) {", "for (int64_t e = 2 * m - 1; e >= 0; e--) {"),
    "window one too wide": ("for (int delta = 1; delta < W; delta++) P += L - delta;",
                            "for (int delta = 1; delta <= W; delta++) P += L - delta;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_fail_on_a_planted_walk_mistake(tmp_path, name):
    find, repl = MUTATIONS[name]
    src = open(ORACLE_C).read()
    assert src.count(find) == 1, name
    c_path = tmp_path / "oracle_mutant.c"
    c_path.write_text(src.replace(find, repl))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c_path), "-lm"])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", os.path.abspath(__file__),
                        "-k", "not planted"], cwd=ROOT, env=dict(os.environ, LH_ORACLE_SO=str(so)),
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.returncode, r.stdout[-2000:])
