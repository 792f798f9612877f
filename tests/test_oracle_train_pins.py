"""Pins of the oracle's training loop (``or_train``) that do not rest on ``or_train`` itself.

The per-sample rule (``apply_tuple``) is pinned elsewhere by finite differences and by the
brute-force expectation over every outcome.  What those leave open is how ``or_train``
strings samples together, and these tests pin it from the definitions:

* the step size of sample s is eta0 (1 - s / T) (linear decay by global sample index, no
  floor), computed here from that formula;
* first-order proximity trains U1 at both ends of the pair, and second order (U, C), on the
  same drawn tuple;
* SEQ applies each sample before the next one is drawn;
* SNAPSHOT(B) (Eq. (4): a row's batch update is the sum of the per-pair contributions
  computed against the copy taken at the start of the batch) groups samples into batches
  [bB, (b+1)B) of the global sample index, also when a run starts inside a batch.

Each pin is then run against copies of the oracle with one plausible mistake planted in
its source (a shifted step-size index, the wrong table in first order, batches aligned to
the run's start): every such copy must fail the pin.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from synth.graphs import Graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")


def _graph(n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m).astype(np.int32)
    dst = rng.integers(0, n, size=m).astype(np.int32)
    w = rng.lognormal(0.0, 1.0, size=m).astype(np.float32)
    return Graph(n=n, src=src, dst=dst, w=w)


def _model(t, d, K, T, lam, alpha, eta0, seed, start_seed):
    m = oracle.Model(t, d=d, K=K, orders=3, T=T, seed=seed, eta0=eta0, lam=lam, alpha=alpha)
    rng = np.random.default_rng(start_seed)
    for X in (m.U, m.C, m.U1):
        X[:] = rng.normal(0.0, 0.5, size=X.shape)
    return m


def _step_size(eta0, s, T):
    # the schedule as defined: linear decay to zero by the global sample index
    return eta0 * (1.0 - s / T)


def _tuple(t, seed, K, s):
    u, v, neg = oracle.sample(t, seed=seed, graph_id=0, K=K, first=s, count=1)
    return int(u[0]), [int(v[0])] + [int(x) for x in neg[0]]


# ---------------------------------------------------------------------------
# SEQ: schedule, both orders, one sample after another.
# ---------------------------------------------------------------------------
SEQ = dict(n=40, m=300, d=8, K=3, T=1000, lam=0.01, alpha=0.7, eta0=0.05, seed=21)


@pytest.mark.parametrize("s", [0, 1, 333, 640, 999])
def test_seq_single_sample_takes_the_scheduled_step_in_both_orders(s):
    c = SEQ
    g = _graph(c["n"], c["m"], 5)
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    m = _model(t, c["d"], c["K"], c["T"], c["lam"], c["alpha"], c["eta0"], c["seed"], 100 + s)
    U, C, U1 = m.U.copy(), m.C.copy(), m.U1.copy()
    m.train(s, 1, "seq")
    u, ids = _tuple(t, c["seed"], c["K"], s)
    eta = _step_size(c["eta0"], s, c["T"])
    oracle.apply_tuple(U, C, u, ids, eta, c["lam"], c["alpha"])      # second order: (U, C)
    oracle.apply_tuple(U1, U1, u, ids, eta, c["lam"], c["alpha"])    # first order: U1 both ends
    assert np.array_equal(m.U, U) and np.array_equal(m.C, C) and np.array_equal(m.U1, U1)


def test_seq_run_applies_samples_in_order():
    c = SEQ
    g = _graph(c["n"], c["m"], 6)
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    m = _model(t, c["d"], c["K"], c["T"], c["lam"], c["alpha"], c["eta0"], c["seed"], 7)
    U, C, U1 = m.U.copy(), m.C.copy(), m.U1.copy()
    first, count = 123, 60
    m.train(first, count, "seq")
    for s in range(first, first + count):
        u, ids = _tuple(t, c["seed"], c["K"], s)
        eta = _step_size(c["eta0"], s, c["T"])
        oracle.apply_tuple(U, C, u, ids, eta, c["lam"], c["alpha"])
        oracle.apply_tuple(U1, U1, u, ids, eta, c["lam"], c["alpha"])
    assert np.array_equal(m.U, U) and np.array_equal(m.C, C) and np.array_equal(m.U1, U1)


# ---------------------------------------------------------------------------
# SNAPSHOT: Eq. (4) with globally aligned batches.
# ---------------------------------------------------------------------------
SNAP = dict(n=5, m=12, d=4, K=2, T=200, lam=0.02, alpha=0.8, eta0=0.2, seed=33)


def _snapshot_by_definition(t, U, C, U1, first, count, B):
    """Batch b covers [bB, (b+1)B) of the global index, cut to [first, first + count).  Every
    sample's increments are taken against the tables frozen at the batch start (as the
    change one sample would make to the frozen copy), summed per row, and added once."""
    c = SNAP
    end = first + count
    s = first
    while s < end:
        b1 = min((s // B + 1) * B, end)
        F = [U.copy(), C.copy(), U1.copy()]
        acc = [np.zeros_like(X) for X in F]
        for q in range(s, b1):
            u, ids = _tuple(t, c["seed"], c["K"], q)
            eta = _step_size(c["eta0"], q, c["T"])
            A2, B2 = F[0].copy(), F[1].copy()
            oracle.apply_tuple(A2, B2, u, ids, eta, c["lam"], c["alpha"])
            acc[0] += A2 - F[0]
            acc[1] += B2 - F[1]
            O2 = F[2].copy()
            oracle.apply_tuple(O2, O2, u, ids, eta, c["lam"], c["alpha"])
            acc[2] += O2 - F[2]
        U += acc[0]
        C += acc[1]
        U1 += acc[2]
        s = b1


@pytest.mark.parametrize("B,first,count", [(1, 0, 25), (3, 10, 20), (7, 10, 30), (7, 14, 21), (64, 5, 150),
                                           (200, 0, 200)])
def test_snapshot_batches_are_eq4_sums_over_global_batches(B, first, count):
    c = SNAP
    rng = np.random.default_rng(B + first)
    src = rng.integers(0, c["n"], size=c["m"]).astype(np.int32)
    dst = rng.integers(0, c["n"], size=c["m"]).astype(np.int32)
    g = Graph(n=c["n"], src=src, dst=dst, w=rng.uniform(0.5, 2.0, size=c["m"]).astype(np.float32))
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    m = _model(t, c["d"], c["K"], c["T"], c["lam"], c["alpha"], c["eta0"], c["seed"], B)
    U, C, U1 = m.U.copy(), m.C.copy(), m.U1.copy()
    m.train(first, count, "snapshot", B)
    _snapshot_by_definition(t, U, C, U1, first, count, B)
    for got, ref in ((m.U, U), (m.C, C), (m.U1, U1)):
        assert np.max(np.abs(got - ref)) <= 1e-12, np.max(np.abs(got - ref))
    # a batch longer than one sample does differ from SEQ on these five rows
    if B > 1:
        s = _model(t, c["d"], c["K"], c["T"], c["lam"], c["alpha"], c["eta0"], c["seed"], B)
        s.train(first, count, "seq")
        assert np.max(np.abs(s.C - m.C)) > 1e-6


# ---------------------------------------------------------------------------
# Planted mistakes: a copy of the oracle with one change must fail the pin it targets.
# ---------------------------------------------------------------------------
MUTATIONS = {
    "step size uses s + 1": (
        "double eta = eta0 * (1.0 - (double)s / (double)T);",
        "double eta = eta0 * (1.0 - (double)(s + 1) / (double)T);",
        ["test_seq_single_sample_takes_the_scheduled_step_in_both_orders",
         "test_snapshot_batches_are_eq4_sums_over_global_batches"]),
    "no decay": (
        "double eta = eta0 * (1.0 - (double)s / (double)T);",
        "double eta = eta0;",
        ["test_seq_single_sample_takes_the_scheduled_step_in_both_orders"]),
    "first order reads U as its vertex table (SEQ)": (
        "double *A = o == 2 ? U : U1, *B = o == 2 ? C : U1;",
        "double *A = o == 2 ? U : U, *B = o == 2 ? C : U1;",
        ["test_seq_single_sample_takes_the_scheduled_step_in_both_orders"]),
    "first order writes C as its context table (SEQ)": (
        "double *A = o == 2 ? U : U1, *B = o == 2 ? C : U1;",
        "double *A = o == 2 ? U : U1, *B = o == 2 ? C : C;",
        ["test_seq_run_applies_samples_in_order"]),
    "first order uses U in SNAPSHOT": (
        "int ta = o == 2 ? 0 : 2, tb = o == 2 ? 1 : 2;",
        "int ta = o == 2 ? 0 : 0, tb = o == 2 ? 1 : 2;",
        ["test_snapshot_batches_are_eq4_sums_over_global_batches"]),
    "batches aligned to the run's first sample": (
        "uint64_t bend = (s / batch + 1) * batch;",
        "uint64_t bend = s + batch;",
        ["test_snapshot_batches_are_eq4_sums_over_global_batches"]),
    "batch rows applied at once (SEQ inside SNAPSHOT)": (
        "for (int c = 0; c < d; c++) acc[ta][(int64_t)u * d + c] += dA[c];",
        "for (int c = 0; c < d; c++) tab[ta][(int64_t)u * d + c] += dA[c];",
        ["test_snapshot_batches_are_eq4_sums_over_global_batches"]),
}


def _build_mutant(tmp_path, find, repl):
    src = open(ORACLE_C).read()
    assert src.count(find) >= 1, f"the planted mistake's target is not in oracle.c: {find}"
    mutated = src.replace(find, repl)
    c_path = tmp_path / "oracle_mutant.c"
    c_path.write_text(mutated)
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c_path), "-lm"])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_fail_on_a_planted_mistake(tmp_path, name):
    find, repl, tests = MUTATIONS[name]
    so = _build_mutant(tmp_path, find, repl)
    env = dict(os.environ, LH_ORACLE_SO=so)
    sel = " or ".join(tests)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.abspath(__file__), "-k", f"({sel}) and not planted"],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    # exit status 1: tests ran and at least one failed (not a crash, not "nothing collected")
    assert r.returncode == 1, (name, r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert " failed" in r.stdout, r.stdout[-2000:]
