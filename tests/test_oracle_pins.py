"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks one part of the oracle against a library routine, exact rational
arithmetic, a textbook algorithm with a different structure, finite differences of
an independently written loss, or a brute-force expectation over every outcome.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle

EPS = np.finfo(np.float64).eps
TWO64 = 1 << 64


# ---------------------------------------------------------------------------
# Philox4x64-10 against numpy's implementation of the same generator.
# ---------------------------------------------------------------------------
def numpy_block(key, ctr):
    """numpy's Philox returns Block(counter + 1); step the counter back by one."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & (TWO64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (1, 0, 0, 0)),
    ((12345, (1 << 32) | 7), (2**40 + 3, 5, 2, 0)),
    ((TWO64 - 1, TWO64 - 1), (TWO64 - 1, TWO64 - 1, TWO64 - 1, TWO64 - 1)),
    ((0xDEADBEEF, 3), (0, 1, 0, 0)),
    ((7, (2 << 32) | 1), (2**33 + 1, 0, 9, 4)),
])
def test_philox_matches_numpy(key, ctr):
    assert np.array_equal(oracle.philox(key, ctr), numpy_block(key, ctr))


def test_philox_many_random_counters():
    rng = np.random.default_rng(0)
    for _ in range(200):
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        assert np.array_equal(oracle.philox(key, ctr), numpy_block(key, ctr))


# ---------------------------------------------------------------------------
# Canonical scan against correctly rounded sums (math.fsum).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 1023, 1024, 1025, 3001, 1024 * 1024 + 17])
def test_cscan_matches_exact_prefix_sums(n):
    rng = np.random.default_rng(n)
    x = rng.lognormal(0.0, 2.0, size=n)
    out = oracle.cscan(x)
    idx = sorted(set([0, n - 1, min(n - 1, 1023), min(n - 1, 1024), n // 2, n // 3]
                     + list(rng.integers(0, n, size=12))))
    for i in idx:
        exact = math.fsum(x[: i + 1])
        assert abs(out[i] - exact) <= 8 * EPS * exact, (i, out[i], exact)


def test_mscan_is_monotone_and_close():
    rng = np.random.default_rng(5)
    x = rng.random(300_000) * (rng.random(300_000) < 0.3)
    c = oracle.cscan(x)
    m = oracle.mscan(x)
    assert np.all(np.diff(m) >= 0)
    assert np.all(m >= c)
    assert np.max(np.abs(m - c)) <= 8 * EPS * c[-1]


# ---------------------------------------------------------------------------
# Alias tables.
# ---------------------------------------------------------------------------
def implied_probabilities(thr, alias):
    """Exact probability of each item under the integer alias table, as Fractions of 1:
    P_i = [thr_i [alias_i != i] + 2^64 [alias_i == i] + sum_{c: alias_c = i, c != i}
    (2^64 - thr_c)] / (N 2^64), where a column keeps itself when x1 < thr."""
    N = len(thr)
    num = [0] * N
    for c in range(N):
        t = int(thr[c])
        a = int(alias[c])
        num[c] += t
        num[a] += TWO64 - t
    return [Fraction(v, N * TWO64) for v in num]


def implied_probabilities_f64(thr, alias):
    N = thr.size
    t = thr.astype(np.float64) / 2.0**64
    t[thr == np.uint64(TWO64 - 1)] = 1.0
    p = t.copy()
    np.add.at(p, alias, 1.0 - t)
    return p / N


def closed_form_exact(w):
    """The closed form of the sweeping alias construction in exact rationals."""
    N = len(w)
    W = sum(w)
    q = [Fraction(x) * N / W for x in w]
    L = [i for i in range(N) if q[i] < 1]
    H = [i for i in range(N) if q[i] >= 1]
    D, acc = [], Fraction(0)
    for i in L:
        acc += 1 - q[i]
        D.append(acc)
    X, acc = [], Fraction(0)
    for i in H:
        acc += q[i] - 1
        X.append(acc)
    S = [Fraction(0)] + D[:-1]
    prob = [Fraction(1)] * N
    alias = list(range(N))
    if H:
        for a, i in enumerate(L):
            k = min(sum(1 for x in X if x <= S[a]), len(H) - 1)
            prob[i], alias[i] = q[i], H[k]
        for k, i in enumerate(H[:-1]):
            j = sum(1 for s in S if s < X[k]) - 1
            o = max(Fraction(0), D[j] - X[k]) if j >= 0 else Fraction(0)
            if o > 0:
                prob[i], alias[i] = max(Fraction(0), 1 - o), H[k + 1]
    return prob, alias


def test_closed_form_reproduces_weights_exactly():
    """The closed form itself (in rationals) must encode w_i / W exactly."""
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(400):
        N = int(rng.integers(1, 12))
        kind = rng.integers(0, 4)
        if kind == 0:
            w = [Fraction(int(x)) for x in rng.integers(0, 6, size=N)]
        elif kind == 1:
            w = [Fraction(int(x), int(y)) for x, y in zip(rng.integers(1, 50, N), rng.integers(1, 9, N))]
        elif kind == 2:  # one dominant item: heavies turn light in a chain
            w = [Fraction(1)] * N
            w[int(rng.integers(0, N))] = Fraction(int(rng.integers(5, 100)))
        else:
            w = [Fraction(int(x)) for x in rng.integers(0, 3, size=N)]
            w[-1] += 1
        if sum(w) == 0:
            w[0] = Fraction(1)
        cases.append(w)
    for w in cases:
        N, W = len(w), sum(w)
        prob, alias = closed_form_exact(w)
        got = [Fraction(0)] * N
        for c in range(N):
            got[c] += prob[c] / N
            got[alias[c]] += (1 - prob[c]) / N
        assert got == [x / W for x in w], w


def alias_error_bound(w, thr, alias):
    """Per-item absolute bound on |P_i - w_i/W| for the binary64 construction.

    Lights: two roundings in q_i, the error of W and the 2^-64 threshold quantum.
    Heavies: additionally the error of the scanned deficit/excess sums that decide the
    overflow o, gamma * D_total per sum involved (compensated chains: gamma = 8 eps),
    plus one quantum per column aliasing to the item."""
    N = w.size
    W = w.sum()
    q = w * N / W
    Dtot = np.sum(np.maximum(0.0, 1.0 - q[q < 1]))
    a_i = np.bincount(alias[alias != np.arange(N)], minlength=N)
    gamma = 8 * EPS
    heavy = q >= 1
    base = (w / W) * 8 * EPS + 2.0**-62 / N
    extra = ((4 + a_i) * gamma * max(Dtot, 1.0) + (1 + a_i) * 2.0**-62) / N
    return base + np.where(heavy | (a_i > 0), extra, 0.0)


@pytest.mark.parametrize("seed", range(12))
def test_oracle_alias_implied_probabilities_small(seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(1, 60))
    w = rng.lognormal(0, 1.5, size=N) * (rng.random(N) < 0.8)
    if w.sum() == 0:
        w[0] = 1.0
    thr, alias = oracle.alias_build(w)
    P = implied_probabilities(thr, alias)
    W = math.fsum(w)
    bound = alias_error_bound(w, thr, alias)
    for i in range(N):
        exact = Fraction(w[i]) / Fraction(W)
        assert abs(float(P[i] - exact)) <= bound[i], (i, float(P[i]), float(exact))


@pytest.mark.parametrize("N", [1000, 200_003])
def test_oracle_alias_implied_probabilities_large(N):
    rng = np.random.default_rng(N)
    w = rng.lognormal(0, 2.0, size=N)
    w[rng.random(N) < 0.05] = 0.0
    thr, alias = oracle.alias_build(w)
    P = implied_probabilities_f64(thr, alias)
    p = w / math.fsum(w)
    bound = alias_error_bound(w, thr, alias) + 4 * EPS * p + 2.0**-60 / N
    assert np.all(np.abs(P - p) <= bound)
    assert np.all(P[w == 0] == 0.0)


def test_alias_bound_catches_plausible_mistakes():
    """A wrong alias target or a dropped overflow must be caught by the bound."""
    rng = np.random.default_rng(3)
    w = rng.lognormal(0, 1.0, size=500)
    thr, alias = oracle.alias_build(w)
    bound = alias_error_bound(w, thr, alias)
    p = w / w.sum()
    heavy_with_overflow = np.where((alias != np.arange(w.size)) &
                                   (w * w.size / w.sum() >= 1))[0]
    assert heavy_with_overflow.size > 0
    bad = alias.copy()
    k = heavy_with_overflow[0]
    bad[k] = k  # overflow dropped
    assert np.any(np.abs(implied_probabilities_f64(thr, bad) - p) > bound)
    light = np.where(w * w.size / w.sum() < 1)[0][0]
    bad = alias.copy()
    bad[light] = (alias[light] + 1) % w.size
    assert np.any(np.abs(implied_probabilities_f64(thr, bad) - p) > bound)


def vose(w):
    """Textbook Vose alias method (stacks, a different pairing)."""
    N = len(w)
    q = [x * N / sum(w) for x in w]
    small = [i for i in range(N) if q[i] < 1]
    large = [i for i in range(N) if q[i] >= 1]
    prob, alias = [1.0] * N, list(range(N))
    while small and large:
        s, l_ = small.pop(), large.pop()
        prob[s], alias[s] = q[s], l_
        q[l_] = (q[l_] + q[s]) - 1
        (small if q[l_] < 1 else large).append(l_)
    return np.array(prob), np.array(alias)


def test_oracle_alias_agrees_with_textbook_vose():
    rng = np.random.default_rng(21)
    for _ in range(20):
        N = int(rng.integers(2, 400))
        w = rng.lognormal(0, 1.0, size=N)
        prob, al = vose(list(w))
        pv = prob.copy()
        np.add.at(pv, al, 1 - prob)
        thr, alias = oracle.alias_build(w)
        assert np.allclose(implied_probabilities_f64(thr, alias), pv / N, rtol=0, atol=1e-12)


def test_alias_special_cases():
    thr, alias = oracle.alias_build(np.ones(37))
    assert np.all(thr == np.uint64(TWO64 - 1)) and np.array_equal(alias, np.arange(37))
    thr, alias = oracle.alias_build(np.array([3.0]))
    assert thr[0] == np.uint64(TWO64 - 1) and alias[0] == 0
    # two items: the light one keeps q = 2 w_l / W and aliases to the heavy one
    thr, alias = oracle.alias_build(np.array([1.0, 3.0]))
    assert int(thr[0]) == TWO64 // 2 and alias[0] == 1
    assert thr[1] == np.uint64(TWO64 - 1) and alias[1] == 1
    # zero weights are never drawn
    thr, alias = oracle.alias_build(np.array([0.0, 2.0, 0.0, 1.0]))
    P = implied_probabilities(thr, alias)
    assert P[0] == 0 and P[2] == 0
    with pytest.raises(ValueError):
        oracle.alias_build(np.zeros(5))


def test_negative_weights_are_degree_power():
    deg = np.concatenate([np.arange(0, 5000), [2**20, 2**26 - 1, 2**30]]).astype(np.int64)
    nu = oracle.neg_weights(deg)
    ref = deg.astype(np.float64) ** 0.75
    assert np.all(np.abs(nu - ref) <= 2 * EPS * ref)
    assert nu[0] == 0.0 and nu[1] == 1.0 and nu[16] == 8.0


# ---------------------------------------------------------------------------
# Draw mapping with crafted words.
# ---------------------------------------------------------------------------
def test_draw_mapping_crafted_words():
    N = 7
    w = np.array([1.0, 2.0, 0.5, 3.0, 0.25, 1.0, 0.25])
    thr, alias = oracle.alias_build(w)
    for k in range(N):
        x0 = -(-k * TWO64 // N)  # ceil(k 2^64 / N) is the first word of column k
        t = int(thr[k])
        if t > 0:
            assert oracle.draw_item(thr, alias, x0, t - 1) == k
        expect = k if t == TWO64 - 1 and alias[k] == k else int(alias[k])
        assert oracle.draw_item(thr, alias, x0, min(t, TWO64 - 1)) == expect
        if k > 0:
            assert oracle.draw_item(thr, alias, x0 - 1, 0) in (k - 1, int(alias[k - 1]))
            assert oracle.draw_item(thr, alias, x0 - 1, 0) == (k - 1 if thr[k - 1] > 0 else alias[k - 1])
    assert oracle.draw_item(thr, alias, 0, 0) == (0 if thr[0] > 0 else alias[0])
    assert oracle.draw_item(thr, alias, TWO64 - 1, 0) == (N - 1 if thr[N - 1] > 0 else alias[N - 1])


# ---------------------------------------------------------------------------
# Frequencies of sampled edges and negatives (chi-square).
# ---------------------------------------------------------------------------
def _binned_chisquare(counts, expected, min_expected=5.0):
    order = np.argsort(expected)
    e, c = expected[order], counts[order]
    keep = e >= min_expected
    e2 = np.concatenate([e[keep], [e[~keep].sum()]]) if (~keep).any() else e[keep]
    c2 = np.concatenate([c[keep], [c[~keep].sum()]]) if (~keep).any() else c[keep]
    nz = e2 > 0
    return stats.chisquare(c2[nz], e2[nz] * c2[nz].sum() / e2[nz].sum()).pvalue


def _arc_index(t, u, v):
    keys = t.src.astype(np.int64) * t.n + t.dst
    order = np.argsort(keys)
    pos = np.searchsorted(keys[order], u.astype(np.int64) * t.n + v)
    return order[pos]


@pytest.mark.slow
def test_edge_frequencies_chisquare(c1_tables):
    t = c1_tables
    T = 10_000_000
    u, v, _ = oracle.sample(t, seed=1, graph_id=0, K=0, first=0, count=T)
    arcs = _arc_index(t, u, v)
    assert np.array_equal(t.src[arcs], u) and np.array_equal(t.dst[arcs], v)
    counts = np.bincount(arcs, minlength=t.m).astype(np.float64)
    expected = t.w.astype(np.float64) / t.w.sum() * T
    assert _binned_chisquare(counts, expected) > 1e-3


@pytest.mark.slow
def test_negative_frequencies_chisquare_and_power(c1_graph):
    g = c1_graph
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    _, _, neg = oracle.sample(t, seed=3, graph_id=0, K=5, first=0, count=2_000_000)
    counts = np.bincount(neg.ravel(), minlength=g.n).astype(np.float64)
    nu = t.deg.astype(np.float64) ** 0.75
    expected = nu / nu.sum() * neg.size
    assert _binned_chisquare(counts, expected) > 1e-3
    assert counts[t.deg == 0].sum() == 0
    # power: a table built from slightly perturbed weights must be rejected
    nu_bad = nu.copy()
    nu_bad[np.argsort(-nu)[:50]] *= 1.05
    thr, alias = oracle.alias_build(nu_bad)
    t.nthr, t.nalias = thr, alias
    _, _, neg2 = oracle.sample(t, seed=3, graph_id=0, K=5, first=0, count=2_000_000)
    counts2 = np.bincount(neg2.ravel(), minlength=g.n).astype(np.float64)
    assert _binned_chisquare(counts2, expected) < 1e-6


@pytest.mark.slow
def test_negative_frequencies_million_node_table():
    rng = np.random.default_rng(8)
    n = 1 << 20
    deg = np.minimum((rng.pareto(1.2, size=n) * 3).astype(np.int64), 50_000)
    src = np.repeat(np.arange(n, dtype=np.int32), deg)
    dst = rng.integers(0, n, size=src.size).astype(np.int32)
    t = oracle.Tables(n, src, dst, np.ones(src.size, dtype=np.float32))
    _, _, neg = oracle.sample(t, seed=9, graph_id=2, K=5, first=2**33, count=2_000_000)
    counts = np.bincount(neg.ravel(), minlength=n).astype(np.float64)
    nu = deg.astype(np.float64) ** 0.75
    assert _binned_chisquare(counts, nu / nu.sum() * neg.size) > 1e-3


# ---------------------------------------------------------------------------
# Gradients: finite differences of the per-sample LINE loss.
# ---------------------------------------------------------------------------
def log_sigmoid(x):
    return -np.logaddexp(0.0, -x)


def sample_loss(A, B, u, ids, lam, alpha):
    """l = -log s(a.b0) - alpha sum_k log s(-a.bk) + lam/2 [(1+K)|a|^2 + sum_j |bj|^2]."""
    a = A[u]
    K = len(ids) - 1
    x = [float(a @ B[r]) for r in ids]
    loss = -log_sigmoid(x[0]) - alpha * sum(log_sigmoid(-xk) for xk in x[1:])
    loss += 0.5 * lam * ((1 + K) * float(a @ a) + sum(float(B[r] @ B[r]) for r in ids))
    return loss


def fd_grad(f, arrays, h=1e-4):
    """4th-order central differences of f with respect to every entry of the arrays."""
    grads = []
    for X in arrays:
        g = np.zeros_like(X)
        it = np.nditer(X, flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = X[i]
            vals = []
            for step in (-2, -1, 1, 2):
                X[i] = old + step * h
                vals.append(f())
            X[i] = old
            g[i] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        grads.append(g)
    return grads


@pytest.mark.parametrize("order,ids,u,lam,alpha", [
    (2, [1, 2, 3], 0, 0.0, 1.0),
    (2, [1, 3, 3, 1], 0, 0.1, 0.5),   # repeated negatives, negative equal to v
    (1, [0, 2, 4], 0, 0.0, 1.0),      # first order, v == u
    (1, [2, 0, 0, 2], 0, 0.05, 2.0),  # first order, negatives repeat u and v
])
def test_update_is_minus_eta_gradient(order, ids, u, lam, alpha):
    rng = np.random.default_rng(len(ids) + order)
    n, d, eta = 6, 8, 0.01
    A = rng.normal(0, 0.5, size=(n, d))
    B = A if order == 1 else rng.normal(0, 0.5, size=(n, d))
    A0, B0 = A.copy(), B.copy()
    if order == 1:
        grads = fd_grad(lambda: sample_loss(A, A, u, ids, lam, alpha), [A])
        oracle.apply_tuple(A, A, u, ids, eta, lam, alpha)
        assert np.allclose(A - A0, -eta * grads[0], rtol=1e-7, atol=1e-12)
    else:
        grads = fd_grad(lambda: sample_loss(A, B, u, ids, lam, alpha), [A, B])
        oracle.apply_tuple(A, B, u, ids, eta, lam, alpha)
        assert np.allclose(A - A0, -eta * grads[0], rtol=1e-7, atol=1e-12)
        assert np.allclose(B - B0, -eta * grads[1], rtol=1e-7, atol=1e-12)


# ---------------------------------------------------------------------------
# SGD on the LINE objective: the expected update over every (arc, negatives)
# outcome equals -eta times the gradient of the expected loss.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K,order,lam", [(1, 2, 0.0), (2, 2, 0.1), (1, 1, 0.0), (2, 1, 0.05)])
def test_expected_update_is_objective_gradient(K, order, lam):
    import itertools
    rng = np.random.default_rng(40 + K + order)
    n, d, eta, alpha = 5, 4, 0.02, 0.7
    src = np.array([0, 1, 2, 3, 0, 4, 2])
    dst = np.array([1, 2, 0, 0, 3, 1, 4])
    w = np.array([1.0, 2.0, 0.5, 1.5, 1.0, 0.25, 3.0])
    p_arc = w / w.sum()
    deg = np.bincount(src, minlength=n).astype(np.float64)
    qn = deg**0.75 / (deg**0.75).sum()
    A = rng.normal(0, 0.4, size=(n, d))
    B = A if order == 1 else rng.normal(0, 0.4, size=(n, d))

    def objective():
        Bt = A if order == 1 else B
        total = 0.0
        for a_, pa in enumerate(p_arc):
            u, v = src[a_], dst[a_]
            total += pa * (-log_sigmoid(A[u] @ Bt[v]) + 0.5 * lam * (1 + K) * (A[u] @ A[u])
                           + 0.5 * lam * (Bt[v] @ Bt[v]))
            for nn in range(n):
                total += pa * K * qn[nn] * (-alpha * log_sigmoid(-(A[u] @ Bt[nn]))
                                            + 0.5 * lam * (Bt[nn] @ Bt[nn]))
        return total

    arrays = [A] if order == 1 else [A, B]
    grads = fd_grad(objective, arrays)
    expA = np.zeros_like(A)
    expB = np.zeros_like(B)
    for a_, pa in enumerate(p_arc):
        for negs in itertools.product(range(n), repeat=K):
            pr = pa * np.prod([qn[x] for x in negs])
            if pr == 0:
                continue
            A2 = A.copy()
            B2 = A2 if order == 1 else B.copy()
            oracle.apply_tuple(A2, B2, int(src[a_]), [int(dst[a_]), *negs], eta, lam, alpha)
            expA += pr * (A2 - A)
            if order == 2:
                expB += pr * (B2 - B)
    assert np.allclose(expA, -eta * grads[0], rtol=1e-8, atol=1e-13)
    if order == 2:
        assert np.allclose(expB, -eta * grads[1], rtol=1e-8, atol=1e-13)


# ---------------------------------------------------------------------------
# AUC, init, modes.
# ---------------------------------------------------------------------------
def test_auc_matches_sklearn():
    from sklearn.metrics import roc_auc_score
    rng = np.random.default_rng(1)
    for _ in range(10):
        pos = np.round(rng.normal(0.5, 1, size=500), 1)  # rounding creates ties
        neg = np.round(rng.normal(0.0, 1, size=700), 1)
        ref = roc_auc_score(np.r_[np.ones(500), np.zeros(700)], np.r_[pos, neg])
        assert abs(oracle.auc(pos, neg) - ref) <= 1e-12


@pytest.mark.parametrize("d", [16, 64, 128, 24])
def test_init_values(d):
    rows, seed, g = 300, 77, 3
    for t in range(3):
        X = oracle.init_table(t, rows, d, seed, g)
        # independent recomputation from numpy's Philox
        for r in (0, 1, rows - 1):
            for c in (0, 3, d - 1):
                word = int(numpy_block((seed, (1 << 32) | g), (r, c // 4, t, 0))[c % 4])
                val = np.float32(((word >> 40) - 2**23) * 2.0**-24 / d)
                assert X[r, c] == val
        assert X.min() >= -0.5 / d and X.max() < 0.5 / d
        if d in (16, 64, 128):
            assert np.all((X.astype(np.float64) * d * 2**24) % 1 == 0)
        assert stats.kstest((X.ravel() * d + 0.5), "uniform").pvalue > 1e-4


def _c1_model(c1_tables, T=20_000, orders=2, d=16):
    return oracle.Model(c1_tables, d=d, K=5, orders=orders, T=T, seed=1)


def test_snapshot_batch1_equals_seq(c1_tables):
    for orders in (2, 1, 3):
        a = _c1_model(c1_tables, orders=orders)
        b = _c1_model(c1_tables, orders=orders)
        a.train(0, 5000, "seq")
        b.train(0, 5000, "snapshot", batch=1)
        for x, y in ((a.U, b.U), (a.C, b.C), (a.U1, b.U1)):
            if x is not None:
                assert np.max(np.abs(x - y)) <= 1e-14


def test_resume_is_exact(c1_tables):
    for mode, B in (("seq", 0), ("snapshot", 256)):
        a = _c1_model(c1_tables, orders=3)
        b = _c1_model(c1_tables, orders=3)
        a.train(0, 8192, mode, B)
        b.train(0, 4096, mode, B)
        b.train(4096, 4096, mode, B)
        for x, y in ((a.U, b.U), (a.C, b.C), (a.U1, b.U1)):
            assert np.array_equal(x, y)


def test_snapshot_large_batch_differs_slightly_from_seq(c1_tables):
    a = _c1_model(c1_tables)
    b = _c1_model(c1_tables)
    a.train(0, 20_000, "seq")
    b.train(0, 20_000, "snapshot", batch=4096)
    diff = np.abs(a.C - b.C).max()
    assert 0 < diff < 0.05 * np.abs(a.C).max()


def test_planted_two_communities_reach_high_auc():
    """Sanity: two dense communities with few cross arcs are separable by the scores."""
    from synth.graphs import Graph
    rng = np.random.default_rng(4)
    n, m = 400, 8000
    comm = np.arange(n) % 2
    src = rng.integers(0, n, size=m)
    same = rng.random(m) < 0.95
    dst = np.where(same, (src + 2 * rng.integers(1, n // 2, size=m)) % n,
                   (src + 2 * rng.integers(0, n // 2, size=m) + 1) % n)
    g = Graph(n=n, src=src.astype(np.int32), dst=dst.astype(np.int32), w=np.ones(m, np.float32))
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    mdl = oracle.Model(t, d=16, K=5, orders=2, T=300_000, seed=9)
    mdl.train(0, 300_000, "seq")
    pu = rng.integers(0, n, size=2000)
    pv = (pu + 2 * rng.integers(1, n // 2, size=2000)) % n   # same community
    nv = (pu + 2 * rng.integers(0, n // 2, size=2000) + 1) % n  # other community
    a = oracle.auc(mdl.scores(pu, pv, 2), mdl.scores(pu, nv, 2))
    assert a > 0.9, a
    assert np.all(comm[pu] == comm[pv])


def test_hogwild_f32_single_thread_tracks_seq(c1_tables):
    """With one thread the binary32 timing mode is the SEQ rule in binary32."""
    t = c1_tables
    m = _c1_model(t, T=50_000)
    U = oracle.init_table(0, t.n, 16, 1, 0)
    C = oracle.init_table(1, t.n, 16, 1, 0)
    oracle.train_hogwild_f32(t, U, C, None, 16, 5, 2, 50_000, 1, 0, 0, 50_000, nthreads=1)
    m.train(0, 50_000, "seq")
    assert np.max(np.abs(U - m.U)) < 1e-5 and np.max(np.abs(C - m.C)) < 1e-5
