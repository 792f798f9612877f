"""Pins of the oracle's pair pool (Sec. IV-C, the Augmented-Pair variant on one process:
walks run only until about sqrt(2 T) pairs are collected, and training draws its pairs
from their recombinations), against facts that do not come from the pool code itself:

* the pool size is the least R >= 2 whose triangle R (R - 1) / 2 holds T, checked
  against the closed form ceil((1 + sqrt(1 + 8 T)) / 2) computed with integer square
  roots;
* the collected pairs are the walk source's first R pairs (the walk source has its own
  pins), across several walk batches;
* sample s's pair is (u_i, v_j) with i, j the column draws of numpy's Philox4x64-10 block
  (seed, graph_id; s, 0, 0, 0) over R columns, at indices past 2^32 too;
* the share of drawn pairs that are edges of the graph matches the exact share over the
  R^2 combinations (binomial bound);
* training one pool sample applies the per-sample rule (pinned by finite differences in
  the edge-sampling pins) to that pair and the sample's negatives; SNAPSHOT with B = 1 is
  SEQ; a SNAPSHOT range gives the same tables in one call or cut at a batch boundary,
  with batches that straddle the oracle's internal pieces; bfloat16 storage writes a
  bfloat16 neighbour of the binary64 step.

Planted mistakes in copies of the oracle (a pool one pair too small, pairs collected from
sample 1 on, one Philox word for both columns, the two columns swapped, pieces cut inside a
SNAPSHOT batch) must fail.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from synth.graphs import Graph

from test_oracle_pins import numpy_block

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")


def _graph(seed, n, m):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m)
    dst = (src + rng.integers(1, n, size=m)) % n
    w = rng.lognormal(0, 1.0, size=m)
    return Graph(n=n, src=src.astype(np.int32), dst=dst.astype(np.int32), w=w.astype(np.float32))


def _walker(g, L=9, W=3, Bw=4):
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    return t, oracle.WalkGraph(t, L=L, W=W, Bw=Bw)


def _closed_form_size(T):
    """ceil((1 + sqrt(1 + 8T)) / 2) with an integer square root (at least 2): equality
    when 1 + 8T is a square (then an odd one); otherwise the root lies strictly between
    isqrt and isqrt + 1."""
    x = 1 + 8 * T
    r = math.isqrt(x)
    if r * r == x:
        R = (1 + r) // 2
    elif r % 2:
        R = (r + 3) // 2
    else:
        R = (r + 2) // 2
    return max(R, 2)


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 6, 7, 10, 11, 45, 46, 999, 1000, 10**6, 2 * 10**8, 10**10, 2**40])
def test_pool_size_is_the_least_triangle_holding_T(T):
    assert oracle.pool_size(T) == _closed_form_size(T)


def test_pool_size_over_a_range():
    for T in range(1, 3000):
        R = oracle.pool_size(T)
        assert R * (R - 1) // 2 >= T and (R == 2 or (R - 1) * (R - 2) // 2 < T), T


def test_collected_pairs_are_the_first_walk_pairs():
    g = _graph(1, 90, 400)
    _, wg = _walker(g)                      # 4 walks of 15 pairs: 60 pairs per walk batch
    for R in (1, 59, 60, 61, 200):
        pu, pv, _, _ = wg.pool(seed=3, graph_id=2, R=R)
        u, v = wg.pairs(seed=3, graph_id=2, first=0, count=R)
        assert np.array_equal(pu, u) and np.array_equal(pv, v), R


@pytest.mark.parametrize("first", [0, 12345, 2**32 - 3, 2**41 + 17])
def test_sample_pairs_come_from_the_philox_column_draws(first):
    g = _graph(2, 70, 300)
    _, wg = _walker(g)
    seed, gid, R = 11, 5, 37
    pu, pv, u, v = wg.pool(seed=seed, graph_id=gid, R=R, first=first, count=64)
    for k in range(64):
        x = numpy_block((seed, gid), (first + k, 0, 0, 0))
        i = (int(x[0]) * R) >> 64
        j = (int(x[1]) * R) >> 64
        assert (u[k], v[k]) == (pu[i], pv[j]), k


def test_pairs_of_any_range_agree():
    g = _graph(3, 60, 250)
    _, wg = _walker(g)
    _, _, u, v = wg.pool(seed=1, graph_id=0, R=50, first=2**33, count=500)
    for off in (0, 1, 255, 490):
        _, _, uu, vv = wg.pool(seed=1, graph_id=0, R=50, first=2**33 + off, count=10)
        assert np.array_equal(uu, u[off:off + 10]) and np.array_equal(vv, v[off:off + 10])


def test_share_of_edges_matches_the_combinations():
    """Recombined pairs are mostly not edges: the share of drawn pairs that are edges of
    the walk graph equals the exact share over the R^2 combinations (4.5 sd)."""
    g = _graph(4, 300, 1200)
    _, wg = _walker(g, L=20, W=2, Bw=8)
    R, N = 40, 200_000
    pu, pv, u, v = wg.pool(seed=9, graph_id=1, R=R, first=0, count=N)
    edges = set(zip(g.src.tolist(), g.dst.tolist())) | set(zip(g.dst.tolist(), g.src.tolist()))
    p = sum((int(a), int(b)) in edges for a in pu for b in pv) / (R * R)
    assert 0.0 < p < 0.5
    got = np.mean([(int(a), int(b)) in edges for a, b in zip(u, v)])
    assert abs(got - p) <= 4.5 * math.sqrt(p * (1 - p) / N), (got, p)


@pytest.mark.parametrize("s", [0, 1, 333, 999])
@pytest.mark.parametrize("orders", [2, 1, 3])
def test_one_pool_sample_applies_the_per_sample_rule(s, orders):
    g = _graph(5, 50, 200)
    t, wg = _walker(g, L=12, W=2, Bw=8)
    K, T, eta0, R = 3, 1000, 0.4, 17
    m = oracle.Model(t, d=8, K=K, orders=orders, T=T, seed=4, eta0=eta0, lam=0.01, alpha=0.7)
    rng = np.random.default_rng(s)
    for X in (m.U, m.C, m.U1):
        if X is not None:
            X[:] = rng.normal(0, 0.3, size=X.shape)
    ref = {k: (None if X is None else X.copy()) for k, X in (("U", m.U), ("C", m.C), ("U1", m.U1))}
    m.train(s, 1, "seq", walks=wg, pool=R)
    _, _, u, v = wg.pool(seed=4, graph_id=0, R=R, first=s, count=1)
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


def test_pool_snapshot_with_batch_one_is_seq():
    g = _graph(6, 120, 600)
    t, wg = _walker(g, L=10, W=2, Bw=16)
    a = oracle.Model(t, d=16, K=2, orders=3, T=5000, seed=6, eta0=0.2)
    b = oracle.Model(t, d=16, K=2, orders=3, T=5000, seed=6, eta0=0.2)
    a.train(37, 3000, "seq", walks=wg, pool=100)
    b.train(37, 3000, "snapshot", 1, walks=wg, pool=100)
    for x, y in ((a.U, b.U), (a.C, b.C), (a.U1, b.U1)):
        assert np.max(np.abs(x - y)) <= 1e-14


def test_pool_snapshot_batches_straddle_the_internal_pieces():
    """B = 3000 does not divide 2^20, so batch [1,047,000, 1,050,000) crosses 2^20.  It
    must still be one SNAPSHOT batch: the sum of its samples' increments (each from the
    per-sample rule on the pre-batch tables) added to the pre-batch tables.  And a range
    gives the same tables in one call or cut at a batch boundary."""
    g = _graph(7, 64, 256)
    t, wg = _walker(g, L=6, W=2, Bw=4)
    T, B, b0 = 1_100_000, 3000, 1_047_000
    R = oracle.pool_size(T)
    eta0, K = 0.05, 1
    c = oracle.Model(t, d=8, K=K, orders=2, T=T, seed=8, eta0=eta0)
    c.train(0, b0, "snapshot", B, walks=wg, pool=R)
    pre = (c.U.copy(), c.C.copy())
    c.train(b0, B, "snapshot", B, walks=wg, pool=R)
    _, _, u, v = wg.pool(seed=8, graph_id=0, R=R, first=b0, count=B)
    neg = oracle.sample_negatives(g.n, t.nthr, t.nalias, seed=8, graph_id=0, K=K, first=b0, count=B)
    dU, dC = np.zeros_like(pre[0]), np.zeros_like(pre[1])
    for k in range(B):
        A, Bt = pre[0].copy(), pre[1].copy()
        ids = np.concatenate([[v[k]], neg[k]]).astype(np.int32)
        oracle.apply_tuple(A, Bt, int(u[k]), ids, eta0 * (1.0 - (b0 + k) / T), 0.0, 1.0)
        dU += A - pre[0]
        dC += Bt - pre[1]
    assert np.max(np.abs(c.U - (pre[0] + dU))) <= 1e-12 and np.max(np.abs(c.C - (pre[1] + dC))) <= 1e-12
    c.train(b0 + B, T - b0 - B, "snapshot", B, walks=wg, pool=R)
    a = oracle.Model(t, d=8, K=K, orders=2, T=T, seed=8, eta0=eta0)
    a.train(0, T, "snapshot", B, walks=wg, pool=R)
    assert np.array_equal(a.U, c.U) and np.array_equal(a.C, c.C)


def _bf16_neighbours(x):
    f = np.float32(x)
    b = f.view(np.uint32)
    lo = np.uint32(b & np.uint32(0xFFFF0000)).view(np.float32)
    if np.uint32(b & np.uint32(0xFFFF)) == 0:
        return float(lo), float(lo)
    hi = np.uint32((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32)
    return float(lo), float(hi)


@pytest.mark.parametrize("s", [0, 77, 500])
def test_one_bf16_pool_sample_lands_next_to_the_binary64_step(s):
    g = _graph(8, 40, 160)
    t, wg = _walker(g, L=8, W=2, Bw=4)
    K, R = 2, 9
    a = oracle.Model(t, d=16, K=K, orders=2, T=1000, seed=3, eta0=0.5, storage="bf16")
    b = oracle.Model(t, d=16, K=K, orders=2, T=1000, seed=3, eta0=0.5)
    rng = np.random.default_rng(s)
    for X, Y in ((a.U, b.U), (a.C, b.C)):
        X[:] = oracle.bf16_rne(rng.normal(0, 0.3, size=X.shape))
        Y[:] = X
    before = (a.U.copy(), a.C.copy())
    a.train(s, 1, "seq", walks=wg, pool=R)
    b.train(s, 1, "seq", walks=wg, pool=R)
    _, _, u, v = wg.pool(seed=3, graph_id=0, R=R, first=s, count=1)
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


# ---------------------------------------------------------------------------
# Planted mistakes.
# ---------------------------------------------------------------------------
MUTATIONS = {
    "pool one pair too small": ("while ((u128)R * (u128)(R - 1) / 2 < (u128)T) R++;",
                                "while ((u128)R * (u128)(R + 1) / 2 < (u128)T) R++;"),
    "collected from sample 1": ("            pu[b * per + i] = bu[i];\n            pv[b * per + i] = bv[i];",
                                "            pu[b * per + i] = bu[i + (i + 1 < per)];\n"
                                "            pv[b * per + i] = bv[i + (i + 1 < per)];"),
    "one word for both columns": ("j = (uint64_t)(((u128)x[1] * R) >> 64);", "j = (uint64_t)(((u128)x[0] * R) >> 64);"),
    "columns swapped": ("    *u = pu[i];\n    *v = pv[j];", "    *u = pu[j];\n    *v = pv[i];"),
    "pieces cut inside a batch": ("if (mode == 1) piece = batch > piece ? batch : (piece / batch) * batch;",
                                  "if (mode == 1) piece = batch > piece ? batch : piece;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_fail_on_a_planted_pool_mistake(tmp_path, name):
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
