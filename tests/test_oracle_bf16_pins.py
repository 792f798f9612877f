"""Pins of the oracle's bfloat16 storage mode (tables held as bfloat16, every written value
stochastically rounded), against facts that do not come from the oracle itself:

* stochastic rounding is unbiased: over all 65,536 patterns of its 16 random bits, the
  rounded values average exactly to the binary32 value being rounded;
* every result is one of the two bfloat16 neighbours of that value, and a value already on
  the bfloat16 grid is returned unchanged for every pattern;
* the stored initial values are the round-to-nearest-even bfloat16 of the binary32 initial
  values, as torch's conversion gives them;
* one training sample in this mode leaves every element it writes once on a bfloat16
  neighbour of the binary64 SEQ result from the same tables, and with a zero step size
  leaves the tables bit for bit as they were.

Planted mistakes (rounding to nearest, truncating, a biased rounding offset) must fail.
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


def _f32(x):
    return float(np.float32(x))


def _bf16_neighbours(x):
    """The two bfloat16 values around binary32(x) (equal when it is on the grid)."""
    f = np.float32(x)
    b = f.view(np.uint32)
    lo = np.uint32(b & np.uint32(0xFFFF0000)).view(np.float32)
    if np.uint32(b & np.uint32(0xFFFF)) == 0:
        return float(lo), float(lo)
    hi = np.uint32((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32)
    return float(lo), float(hi)


VALUES = [0.1, -0.1, 1.0 / 3.0, -2.0 / 3.0, 1e-3, 3.14159, -123.456, 7.7e-20, 6.0e4, 0.0078125 * 1.37]


@pytest.mark.parametrize("x", VALUES)
def test_stochastic_rounding_is_unbiased_over_every_bit_pattern(x):
    vals = np.array([oracle.sr_bf16(x, r) for r in range(65536)])
    lo, hi = _bf16_neighbours(x)
    assert set(np.unique(vals)) <= {lo, hi}
    # the mean over every pattern is the binary32 value itself (up to the float64 sum)
    assert abs(vals.mean() - _f32(x)) <= 1e-15 * abs(_f32(x))


def test_values_on_the_grid_are_kept():
    rng = np.random.default_rng(0)
    for _ in range(200):
        bits = np.uint32(rng.integers(0, 2**16) << 16) & np.uint32(0x7F7FFFFF)
        v = float(np.uint32(bits).view(np.float32)) * rng.choice([-1.0, 1.0])
        for r in (0, 1, 0x7FFF, 0x8000, 0xFFFF):
            assert oracle.sr_bf16(v, r) == v


def test_nearest_rounding_of_initial_values_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 100_000), rng.uniform(-0.004, 0.004, 100_000)]).astype(np.float32)
    # exact ties: a binary32 pattern whose low 16 bits are 0x8000, with odd and even high halves
    ties = (np.arange(1000, dtype=np.uint32) << np.uint32(16)) | np.uint32(0x8000) | np.uint32(0x3F000000)
    x = np.concatenate([x, ties.view(np.float32)])
    ref = torch.tensor(x).to(torch.bfloat16).double().numpy()
    assert np.array_equal(oracle.bf16_rne(x.astype(np.float64)), ref)


def _one_sample_case(eta0):
    rng = np.random.default_rng(5)
    n, m, d, K = 30, 200, 16, 3
    src = rng.integers(0, n, size=m).astype(np.int32)
    dst = rng.integers(0, n, size=m).astype(np.int32)
    g = Graph(n=n, src=src, dst=dst, w=rng.uniform(0.5, 2.0, size=m).astype(np.float32))
    t = oracle.Tables(g.n, g.src, g.dst, g.w)
    a = oracle.Model(t, d=d, K=K, orders=3, T=1000, seed=4, eta0=eta0, storage="bf16")
    b = oracle.Model(t, d=d, K=K, orders=3, T=1000, seed=4, eta0=eta0)
    for X, Y in ((a.U, b.U), (a.C, b.C), (a.U1, b.U1)):
        X[:] = oracle.bf16_rne(rng.normal(0, 0.3, size=X.shape))
        Y[:] = X
    return t, a, b


@pytest.mark.parametrize("s", [0, 17, 400])
def test_one_bf16_sample_lands_next_to_the_binary64_step(s):
    t, a, b = _one_sample_case(eta0=0.5)
    before = [a.U.copy(), a.C.copy(), a.U1.copy()]
    a.train(s, 1, "seq")
    b.train(s, 1, "seq")
    u, v, neg = oracle.sample(t, seed=4, graph_id=0, K=3, first=s, count=1)
    ids = [int(v[0])] + [int(x) for x in neg[0]]
    u = int(u[0])
    checked = 0
    for (X, Y, X0), rows, in zip(((a.U, b.U, before[0]), (a.C, b.C, before[1]), (a.U1, b.U1, before[2])),
                                 ([u], ids, [u] + ids)):
        for r in set(rows):
            if rows.count(r) != 1:
                continue  # written twice in this sample: rounded twice
            for c in range(X.shape[1]):
                lo, hi = _bf16_neighbours(Y[r, c])
                assert X[r, c] in (lo, hi), (r, c, X[r, c], Y[r, c])
                checked += 1
        untouched = np.setdiff1d(np.arange(X.shape[0]), rows)
        assert np.array_equal(X[untouched], X0[untouched])
    assert checked >= 3 * 16


def test_zero_step_leaves_bf16_tables_unchanged():
    t, a, _ = _one_sample_case(eta0=0.0)
    before = [a.U.copy(), a.C.copy(), a.U1.copy()]
    a.train(0, 500, "seq")
    for x, y in zip(before, (a.U, a.C, a.U1)):
        assert np.array_equal(x, y)


MUTATIONS = {
    "rounds to nearest": ("u = (u + (uint32_t)r) & 0xffff0000u;",
                          "u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u; (void)r;"),
    "truncates": ("u = (u + (uint32_t)r) & 0xffff0000u;", "u = u & 0xffff0000u; (void)r;"),
    "biased offset": ("u = (u + (uint32_t)r) & 0xffff0000u;", "u = (u + ((uint32_t)r | 1u)) & 0xffff0000u;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_fail_on_a_planted_rounding_mistake(tmp_path, name):
    find, repl = MUTATIONS[name]
    src = open(ORACLE_C).read()
    assert src.count(find) == 1
    c_path = tmp_path / "oracle_mutant.c"
    c_path.write_text(src.replace(find, repl))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c_path), "-lm"])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", os.path.abspath(__file__),
                        "-k", "unbiased and not planted"], cwd=ROOT, env=dict(os.environ, LH_ORACLE_SO=str(so)),
                       capture_output=True, text=True)
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.returncode, r.stdout[-2000:])
