"""Seeded synthetic graphs with the shapes of the workloads the method is measured on.

Every array is produced by ``numpy.random.default_rng(seed)`` (PCG64), so a given seed
gives the same graph on every machine with the same numpy.  The recipe:

* R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with quadrant probabilities
  (a, b, c, d) = (0.57, 0.19, 0.19, 0.05).  One uniform draw per level picks the
  quadrant; bit ``l`` of the source is set for quadrants c, d and bit ``l`` of the
  destination for quadrants b, d.
* Self-loops and IDs >= n are rejected, duplicates are dropped keeping the first
  occurrence (generation order), and generation continues until exactly ``m`` unique
  edges exist.  For an undirected graph the pair is canonicalised to (min, max) for
  de-duplication and stored as two arcs, (u, v) then (v, u).
* Vertex IDs are relabelled with a seeded random permutation so that hubs are spread
  over the tables instead of sitting at low IDs.
* Weights are 1 (unit) or lognormal(mu=0, sigma=1) rounded to float32, one draw per
  unique edge (both arcs of an undirected edge share it).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

RMAT_ABC = (0.57, 0.19, 0.19)


@dataclass
class Graph:
    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    w: np.ndarray  # float32[m]
    directed: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _rmat_keys(rng, scale: int, n: int, count: int, directed: bool, abc=RMAT_ABC):
    """Draw ``count`` R-MAT pairs, reject out-of-range IDs and self-loops, return keys."""
    a, b, c = abc
    ab, abc_ = a + b, a + b + c
    u = np.zeros(count, dtype=np.int64)
    v = np.zeros(count, dtype=np.int64)
    for lvl in range(scale):
        r = rng.random(count)
        sbit = r >= ab
        dbit = ((r >= a) & (r < ab)) | (r >= abc_)
        u |= sbit.astype(np.int64) << lvl
        v |= dbit.astype(np.int64) << lvl
    keep = (u < n) & (v < n) & (u != v)
    u, v = u[keep], v[keep]
    if not directed:
        lo, hi = np.minimum(u, v), np.maximum(u, v)
        u, v = lo, hi
    return u * n + v


def rmat_graph(scale: int, n: int, m_unique: int, seed: int, directed: bool = True,
               weights: str = "lognormal", abc=RMAT_ABC, relabel: bool = True) -> Graph:
    """R-MAT graph with exactly ``m_unique`` unique edges (see module docstring)."""
    if n > (1 << scale):
        raise ValueError("n exceeds 2**scale")
    rng = np.random.default_rng(seed)
    keys = np.empty(0, dtype=np.int64)
    need = m_unique
    while True:
        batch = int(need * 1.3) + 4096
        fresh = _rmat_keys(rng, scale, n, batch, directed, abc)
        allk = np.concatenate([keys, fresh])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first]
        if keys.shape[0] >= m_unique:
            keys = keys[:m_unique]
            break
        need = m_unique - keys.shape[0]
    u = (keys // n).astype(np.int64)
    v = (keys % n).astype(np.int64)
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        u, v = perm[u], perm[v]
    if weights == "unit":
        w = np.ones(m_unique, dtype=np.float32)
    elif weights == "lognormal":
        w = rng.lognormal(0.0, 1.0, size=m_unique).astype(np.float32)
    else:
        raise ValueError(weights)
    if directed:
        src, dst, ww = u, v, w
    else:
        src = np.empty(2 * m_unique, dtype=np.int64)
        dst = np.empty(2 * m_unique, dtype=np.int64)
        src[0::2], dst[0::2] = u, v
        src[1::2], dst[1::2] = v, u
        ww = np.repeat(w, 2)
    return Graph(n=n, src=src.astype(np.int32), dst=dst.astype(np.int32),
                 w=np.ascontiguousarray(ww, dtype=np.float32), directed=directed,
                 meta=dict(kind="rmat", scale=scale, seed=seed, m_unique=m_unique))


def holdout_split(g: Graph, seed: int, frac_den: int = 100):
    """Hold out exactly floor(m / frac_den) arcs, chosen by ``seed``.

    Returns (train_graph, held_src, held_dst).  The training graph keeps the
    remaining arcs in their original order."""
    rng = np.random.default_rng(seed)
    k = g.m // frac_den
    idx = np.sort(rng.choice(g.m, size=k, replace=False))
    mask = np.ones(g.m, dtype=bool)
    mask[idx] = False
    train = Graph(n=g.n, src=g.src[mask].copy(), dst=g.dst[mask].copy(), w=g.w[mask].copy(),
                  directed=g.directed, meta=dict(g.meta, held_out=k))
    return train, g.src[idx].copy(), g.dst[idx].copy()


def auc_negatives(n: int, all_src: np.ndarray, all_dst: np.ndarray, held_src: np.ndarray,
                  seed: int) -> np.ndarray:
    """One negative endpoint per held-out arc (u, v): v' uniform on [0, n) minus {u},
    redrawn while (u, v') is an arc of the full graph (training plus held-out)."""
    rng = np.random.default_rng(seed)
    ekeys = np.sort(all_src.astype(np.int64) * n + all_dst.astype(np.int64))
    u = held_src.astype(np.int64)
    out = np.empty(u.shape[0], dtype=np.int64)
    todo = np.arange(u.shape[0])
    while todo.size:
        cand = rng.integers(0, n - 1, size=todo.size)
        cand = cand + (cand >= u[todo])
        key = u[todo] * n + cand
        pos = np.searchsorted(ekeys, key)
        pos = np.minimum(pos, ekeys.size - 1)
        bad = ekeys[pos] == key
        out[todo[~bad]] = cand[~bad]
        todo = todo[bad]
    return out.astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads.  C1 is the small correctness case, C2/C3 the headline
# d=128 case, C4 the batched case and C5 the large single-GPU share.
# ---------------------------------------------------------------------------
CONFIGS = {
    "C1": dict(scale=14, n=10_000, m_unique=100_000, seed=1, directed=False, weights="unit",
               d=16, K=5, T=1_000_000, eta0=0.025, orders=2, dtype="fp32"),
    "C2": dict(scale=20, n=1 << 20, m_unique=1 << 24, seed=2, directed=True, weights="lognormal",
               d=128, K=5, T=200_000_000, eta0=0.025, orders=3, dtype="fp32", holdout=True),
    "C3": dict(scale=20, n=1 << 20, m_unique=1 << 24, seed=2, directed=True, weights="lognormal",
               d=128, K=5, T=200_000_000, eta0=0.025, orders=3, dtype="bf16", holdout=True),
    "C5": dict(scale=26, n=1 << 26, m_unique=1 << 30, seed=5, directed=True, weights="lognormal",
               d=128, K=5, T=10_000_000_000, eta0=0.025, orders=2, dtype="bf16"),
    # Uniform-endpoint control at C5's shape (raw random gather/scatter, no hub reuse).
    "C5U": dict(n=1 << 26, m_unique=1 << 30, seed=55, directed=True, weights="unit",
                d=128, K=5, T=10_000_000_000, eta0=0.025, orders=2, dtype="bf16"),
}


def config_graph(name: str, holdout: Optional[bool] = None):
    """Training graph of a named workload.

    Returns ``(train, held_src, held_dst, neg_dst)``; the last three are None when the
    workload has no hold-out.  ``holdout=True`` on C1 gives its 1 % AUC variant."""
    cfg = CONFIGS[name]
    g = rmat_graph(cfg["scale"], cfg["n"], cfg["m_unique"], cfg["seed"], cfg["directed"],
                   cfg["weights"])
    g.meta["config"] = name
    if holdout is None:
        holdout = bool(cfg.get("holdout", False))
    if not holdout:
        return g, None, None, None
    train, hs, hd = holdout_split(g, seed=cfg["seed"] * 1000 + 7)
    neg = auc_negatives(g.n, g.src, g.dst, hs, seed=cfg["seed"] * 1000 + 11)
    return train, hs, hd, neg


def batch_graph_specs(G: int = 64, base_seed: int = 4000, n_lo: float = 1e3, n_hi: float = 2e6,
                      deg_lo: float = 8.0, deg_hi: float = 32.0):
    """Sizes of the batched workload: per graph g, seed base_seed+g draws
    n_g = round(exp(U(ln n_lo, ln n_hi))), mean out-degree U[deg_lo, deg_hi],
    m_g = round(n_g * deg), d_g in {64, 128} with probability 1/2, R-MAT scale
    ceil(log2 n_g)."""
    specs = []
    for gi in range(G):
        rng = np.random.default_rng(base_seed + gi)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        deg = float(rng.uniform(deg_lo, deg_hi))
        m = int(round(n * deg))
        d = int(rng.choice([64, 128]))
        scale = max(1, int(math.ceil(math.log2(n))))
        specs.append(dict(g=gi, seed=base_seed + gi, n=n, m=m, d=d, scale=scale, T=20 * m))
    return specs


def rmat_graph_gpu(scale: int, n: int, m_unique: int, seed: int, weights: str = "lognormal",
                   abc=RMAT_ABC, device: str = "cuda"):
    """Directed R-MAT graph built on the GPU with torch (for graphs too large for numpy,
    e.g. 2^30 arcs).  Same recipe as ``rmat_graph`` (quadrant draws per level, rejection
    of self-loops and IDs >= n, first occurrence kept, exact m, seeded relabelling,
    lognormal weights), with torch's seeded CUDA generator as the source of randomness.
    Returns torch tensors (src int32, dst int32, w float32) on ``device``."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    a, b, c = abc
    keys = torch.empty(0, dtype=torch.int64, device=device)
    need = m_unique
    chunk = 1 << 27
    while True:
        parts = []
        todo = int(need * 1.15) + 4096
        while todo > 0:
            cnt = min(chunk, todo)
            u = torch.zeros(cnt, dtype=torch.int64, device=device)
            v = torch.zeros(cnt, dtype=torch.int64, device=device)
            for lvl in range(scale):
                r = torch.rand(cnt, generator=gen, device=device)
                sbit = r >= (a + b)
                dbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
                u |= sbit.to(torch.int64) << lvl
                v |= dbit.to(torch.int64) << lvl
                del r, sbit, dbit
            keep = (u < n) & (v < n) & (u != v)
            parts.append((u[keep] * n + v[keep]))
            del u, v, keep
            todo -= cnt
        allk = torch.cat([keys] + parts)
        del parts
        # keep the first occurrence of every key, in generation order
        sk, order = torch.sort(allk, stable=True)
        first = torch.ones_like(sk, dtype=torch.bool)
        first[1:] = sk[1:] != sk[:-1]
        idx = torch.sort(order[first]).values
        del sk, order, first
        keys = allk[idx]
        del allk, idx
        if keys.numel() >= m_unique:
            keys = keys[:m_unique]
            break
        need = m_unique - keys.numel()
    perm = torch.randperm(n, generator=gen, device=device)
    src = perm[keys // n].to(torch.int32)
    dst = perm[keys % n].to(torch.int32)
    del keys, perm
    if weights == "unit":
        w = torch.ones(m_unique, dtype=torch.float32, device=device)
    else:
        w = torch.empty(m_unique, dtype=torch.float32, device=device).log_normal_(0.0, 1.0, generator=gen)
    return src, dst, w


def uniform_graph_gpu(n: int, m: int, seed: int, device: str = "cuda"):
    """Control graph with uniformly random endpoints: m arcs, src uniform on [0, n), dst
    uniform on [0, n) minus src (no self-loops; repeated arcs are kept, about m^2 / (2 n^2)
    of them), unit weights.  Out-degrees are then binomial(m, 1/n), so the negative
    distribution deg^0.75 is close to uniform too: rows are touched at near-equal rates and
    no row is a hub.  Built on the GPU with torch's seeded generator; returns (src int32,
    dst int32, w float32) on ``device``."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    src = torch.randint(0, n, (m,), generator=gen, device=device, dtype=torch.int64)
    off = torch.randint(1, n, (m,), generator=gen, device=device, dtype=torch.int64)
    dst = ((src + off) % n).to(torch.int32)
    del off
    src = src.to(torch.int32)
    w = torch.ones(m, dtype=torch.float32, device=device)
    return src, dst, w


def batch_graph(spec: dict) -> Graph:
    """One graph of the batched workload from its spec (directed R-MAT, lognormal)."""
    g = rmat_graph(spec["scale"], spec["n"], spec["m"], spec["seed"] + 100_000, True, "lognormal")
    g.meta.update(spec)
    return g


def small_batch(G: int = 6):
    """A few small graphs for tests of the batched launch: graph gi has n drawn from
    U[2000, 20000), m = n * U[8, 16) unique directed R-MAT arcs (seed 700 + gi), unit
    weights, d = 64 for even gi and 128 for odd gi, a 1 % held-out split (seed 800 + gi)
    with evaluation negatives (seed 900 + gi), T = 20 training epochs, training seed
    10 + gi and graph id gi.  Returns one dict per graph."""
    rng = np.random.default_rng(0)
    out = []
    for gi in range(G):
        n = int(rng.integers(2000, 20000))
        m = int(n * rng.uniform(8, 16))
        g = rmat_graph(int(np.ceil(np.log2(n))), n, m, seed=700 + gi)
        tr, hs, hd = holdout_split(g, seed=800 + gi)
        neg = auc_negatives(g.n, g.src, g.dst, hs, seed=900 + gi)
        out.append(dict(graph=tr, held_src=hs, held_dst=hd, neg_dst=neg, T=20 * tr.m,
                        d=64 if gi % 2 == 0 else 128, seed=10 + gi, graph_id=gi))
    return out


def mid_graph():
    """A mid-size workload whose tables are a few times the GPU's total L2 (where rows written
    by one XCD are most often read by another): directed R-MAT scale 18 restricted to
    150,000 nodes, 1,500,000 unique arcs (seed 41), unit weights, a 1 % held-out split
    (seed 42) with evaluation negatives (seed 43); d = 64, K = 5, second order, 10 epochs
    (T = 10 m), training seed 7.  Returns a dict like small_batch's entries."""
    g = rmat_graph(18, 150_000, 1_500_000, seed=41)
    tr, hs, hd = holdout_split(g, seed=42)
    neg = auc_negatives(g.n, g.src, g.dst, hs, seed=43)
    return dict(graph=tr, held_src=hs, held_dst=hd, neg_dst=neg, T=10 * tr.m, d=64, seed=7, graph_id=0)
