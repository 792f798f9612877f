"""lh_build_alias_noalloc (the alias build for callers that cannot allocate: its scratch is
a static per-GPU array) against lh_build_alias (scratch from the caller): bit-identical
alias tables and sampled tuples, on two calls in a row, the second on a smaller graph, and
a graph beyond the array's size refused before any GPU work."""
import ctypes

import numpy as np
import pytest

from synth import rmat_graph
from synth.graphs import Graph

from gpu_util import trainer_for

pytestmark = pytest.mark.gpu


def _lh():
    import paper_2604_09419_amd as lh
    return lh


def _tables(tr):
    lh = _lh()
    return [tr.export_alias(w) for w in (lh.LH_ALIAS_EDGE, lh.LH_ALIAS_NEG)]


def _noalloc_build(tr):
    """The allocation-free build through the C ABI (no scratch tensor is made)."""
    from paper_2604_09419_amd import _lib
    _lib.lh_build_alias_noalloc(tr.h)


@pytest.mark.parametrize("graphs", [((14, 10_000, 100_000, False), (12, 3_000, 30_000, True))])
def test_noalloc_build_matches_the_scratch_build_twice(graphs):
    for call, (scale, n, m, directed) in enumerate(graphs):
        g = rmat_graph(scale, n, m, seed=60 + call, directed=directed)
        ref = trainer_for(g, d=16, K=5, orders=2, seed=9, total_samples=1000)
        got = trainer_for(g, d=16, K=5, orders=2, seed=9, total_samples=1000, build=False, init=False)
        _noalloc_build(got)
        print(f"call {call}: n={g.n} m={g.m}", flush=True)
        for (t1, a1), (t2, a2) in zip(_tables(ref), _tables(got)):
            assert np.array_equal(t1, t2) and np.array_equal(a1, a2)
        assert got.kernel_config() == ref.kernel_config()
        for first in (0, 2**33 + 1):
            u1, v1, n1 = ref.sample(first, 5000)
            u2, v2, n2 = got.sample(first, 5000)
            assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in ((u1, u2), (v1, v2), (n1, n2)))
        ref.close()
        got.close()


def _random_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    return Graph(n=n, src=rng.integers(0, n, m).astype(np.int32), dst=rng.integers(0, n, m).astype(np.int32),
                 w=rng.lognormal(0.0, 1.0, m).astype(np.float32))


def test_noalloc_build_at_its_largest_size():
    """n = m = 2^21, the largest graph the static scratch takes: equal to the scratch build."""
    g = _random_graph(1 << 21, 1 << 21, 4)
    ref = trainer_for(g, d=8, K=5, orders=2, seed=9, total_samples=10, init=False)
    got = trainer_for(g, d=8, K=5, orders=2, seed=9, total_samples=10, build=False, init=False)
    _noalloc_build(got)
    for (t1, a1), (t2, a2) in zip(_tables(ref), _tables(got)):
        assert np.array_equal(t1, t2) and np.array_equal(a1, a2)


@pytest.mark.parametrize("n,m", [(1000, (1 << 21) + 1), ((1 << 21) + 1, 1000)])
def test_noalloc_build_refuses_graphs_beyond_its_scratch(n, m):
    lh = _lh()
    g = _random_graph(n, m, 3)
    tr = trainer_for(g, d=8, total_samples=10, build=False, init=False)
    with pytest.raises(lh.LhError) as e:
        _noalloc_build(tr)
    assert e.value.status == 1 and "too large" in str(e.value)
    assert _lh()._lib.lib().lh_build_alias_noalloc(None) == 1
    # the handle still builds with a caller's scratch
    tr.build_alias()
    tr.check()
