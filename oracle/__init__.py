"""CPU oracle for LINE-style edge-sampled SGD -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct reference (``oracle.c``, binary64) that the GPU
library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with the
GPU library and imports nothing from it.

Every function cites the passage of the paper (NOMAD, arXiv 2604.09419) it follows;
the C source holds the full statement of each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (no contraction, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = f"{_SO}.{os.getpid()}.tmp"  # processes that build at once each write their own file
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    """The oracle's shared library.  ``LH_ORACLE_SO`` names another build of the same
    source to load instead (the tests use it to run a pin against a copy of the oracle
    with a deliberately planted mistake)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LH_ORACLE_SO")
        if not path:
            build()
            path = _SO
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, u64, u32, i32, f64 = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_int, ctypes.c_double)
        L.or_philox4x64_10.argtypes = [u64, u64, P, P]
        L.or_cscan.argtypes = [P, i64, P]
        L.or_mscan.argtypes = [P, i64, P]
        L.or_out_degree.argtypes = [P, i64, i64, P]
        L.or_neg_weights.argtypes = [P, i64, P]
        L.or_alias_build.argtypes = [P, i64, P, P]
        L.or_alias_build.restype = i32
        L.or_sample.argtypes = [i64, i64, P, P, P, P, P, P, u64, u32, i32, u64, u64, P, P, P]
        L.or_sample_negatives.argtypes = [i64, P, P, u64, u32, i32, u64, u64, P]
        L.or_init_table.argtypes = [P, i32, i64, i32, u64, u32]
        L.or_train.argtypes = [P, P, i64, i64, P, P, P, P, u64, u32, i32, i32, i32,
                               f64, f64, f64, u64, P, P, P, u64, u64, i32, u64]
        L.or_train.restype = i32
        L.or_train_bf16.argtypes = [P, P, i64, i64, P, P, P, P, u64, u32, i32, i32, i32,
                                    f64, f64, f64, u64, P, P, P, u64, u64, u64]
        L.or_train_bf16.restype = i32
        L.or_sr_bf16.argtypes = [f64, u32]
        L.or_sr_bf16.restype = f64
        L.or_bf16_rne.argtypes = [P, i64]
        L.or_train_hogwild_f32.argtypes = [P, P, i64, i64, P, P, P, P, u64, u32, i32, i32, i32,
                                           f64, f64, f64, u64, P, P, P, u64, u64, i32]
        L.or_train_hogwild_f32.restype = i32
        L.or_max_threads.restype = i32
        L.or_auc.argtypes = [P, i64, P, i64]
        L.or_auc.restype = f64
        L.or_pair_scores.argtypes = [P, P, i32, P, P, i64, P]
        L.or_draw_item.argtypes = [P, P, i64, u64, u64]
        L.or_draw_item.restype = i64
        L.or_apply_tuple.argtypes = [P, P, i32, i32, i32, P, f64, f64, f64]
        if hasattr(L, "or_walk_csr"):
            L.or_walk_csr.argtypes = [i64, i64, P, P, P, P, P, P]
            L.or_walk_csr.restype = i32
            L.or_walk_alias.argtypes = [i64, P, P, P, P]
            L.or_walk_pairs.argtypes = [i64, i64, P, P, P, P, P, P, P, P, u64, u32, i32, i32, i64,
                                        u64, u64, P, P]
            L.or_walk_pairs.restype = i32
            L.or_walk_vertices.argtypes = [i64, i64, P, P, P, P, P, P, P, P, u64, u32, i32, u64, u64, P]
            L.or_walk_vertices.restype = i32
            L.or_train_walk.argtypes = [P, P, i64, i64, P, P, P, P, P, P, P, P, i32, i32, i64, u64, u32,
                                        i32, i32, i32, f64, f64, f64, u64, P, P, P, u64, u64, i32, u64]
            L.or_train_walk.restype = i32
            L.or_train_bf16_walk.argtypes = [P, P, i64, i64, P, P, P, P, P, P, P, P, i32, i32, i64, u64,
                                             u32, i32, i32, i32, f64, f64, f64, u64, P, P, P, u64, u64, u64]
            L.or_train_bf16_walk.restype = i32
            L.or_pool_size.argtypes = [u64]
            L.or_pool_size.restype = u64
            L.or_pool_pairs.argtypes = [i64, i64, P, P, P, P, P, P, P, P, u64, u32, i32, i32, i64, u64,
                                        P, P, u64, u64, P, P]
            L.or_pool_pairs.restype = i32
            L.or_train_pool.argtypes = [P, P, i64, i64, P, P, P, P, P, P, P, P, i32, i32, i64, u64, u64,
                                        u32, i32, i32, i32, f64, f64, f64, u64, P, P, P, u64, u64, i32,
                                        u64, i64]
            L.or_train_pool.restype = i32
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# Counter-based generator: Philox4x64-10 (Salmon et al., SC'11).
# --------------------------------------------------------------------------
def philox(key, ctr) -> np.ndarray:
    """One Philox4x64-10 block for key (2 words) and counter (4 words)."""
    c = _c(ctr, np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(int(key[0]), int(key[1]), _p(c), _p(out))
    return out


# --------------------------------------------------------------------------
# Canonical FP64 scan and alias tables (encoding of the discrete distributions of
# Eq. (1) and of Algorithm 3's root-edge selection).
# --------------------------------------------------------------------------
def cscan(x) -> np.ndarray:
    x = _c(x, np.float64)
    out = np.zeros_like(x)
    lib().or_cscan(_p(x), x.size, _p(out))
    return out


def mscan(x) -> np.ndarray:
    x = _c(x, np.float64)
    out = np.zeros_like(x)
    lib().or_mscan(_p(x), x.size, _p(out))
    return out


def out_degree(src, n: int) -> np.ndarray:
    """d(v) of Eq. (1): number of arcs leaving v."""
    s = _c(src, np.int32)
    deg = np.zeros(n, dtype=np.int64)
    lib().or_out_degree(_p(s), s.size, n, _p(deg))
    return deg


def neg_weights(deg) -> np.ndarray:
    """Eq. (1) numerator d(v)^0.75, as sqrt(d) * sqrt(sqrt(d)) in binary64."""
    d = _c(deg, np.int64)
    out = np.zeros(d.size, dtype=np.float64)
    lib().or_neg_weights(_p(d), d.size, _p(out))
    return out


def alias_build(w):
    """Alias table (thr uint64[N], alias int32[N]) for weights w (float64)."""
    w = _c(w, np.float64)
    thr = np.zeros(w.size, dtype=np.uint64)
    al = np.zeros(w.size, dtype=np.int32)
    rc = lib().or_alias_build(_p(w), w.size, _p(thr), _p(al))
    if rc != 0:
        raise ValueError("total weight is zero or not finite")
    return thr, al


def draw_item(thr, alias, x0: int, x1: int) -> int:
    """Item chosen by the words (x0, x1): col = floor(x0 N / 2^64), then the alias test."""
    thr = _c(thr, np.uint64)
    alias = _c(alias, np.int32)
    return int(lib().or_draw_item(_p(thr), _p(alias), thr.size, x0, x1))


def apply_tuple(A, B, u: int, ids, eta: float, lam: float = 0.0, alpha: float = 1.0):
    """Apply one sample (u; v = ids[0]; negatives ids[1:]) to float64 tables A, B in place
    (Algorithm 1 local updates with LineUpdate, Eqs. (2)-(3)).  A and B may be the same
    array (first-order proximity)."""
    ids = _c(ids, np.int32)
    assert A.dtype == np.float64 and A.flags.c_contiguous
    assert B.dtype == np.float64 and B.flags.c_contiguous
    lib().or_apply_tuple(_p(A), _p(B), A.shape[1], ids.size - 1, u, _p(ids), eta, lam, alpha)


class Tables:
    """Edge table over arcs (weights w) and negative table over nodes (Eq. (1))."""

    def __init__(self, n: int, src, dst, w, progress=None):
        """``progress``, if given, is called with a short message after each step (large
        graphs take minutes)."""
        say = progress or (lambda msg: None)
        self.n = int(n)
        self.src = _c(src, np.int32)
        self.dst = _c(dst, np.int32)
        self.w = _c(w, np.float32)
        self.m = int(self.src.size)
        self.deg = out_degree(self.src, self.n)
        say("out-degrees")
        self.ethr, self.ealias = alias_build(self.w.astype(np.float64))
        say("edge alias table")
        self.nthr, self.nalias = alias_build(neg_weights(self.deg))
        say("negative alias table")


class WalkGraph:
    """The random-walk pair source (Sec. IV-B, Algorithms 2-3) over the undirected graph of
    ``tables``' arcs: CSR rows of the neighbourhoods N(x) (entry e < m is arc e forwards,
    m + e arc e backwards, in entry order within a row), the per-row alias tables of
    discrete(N(x)), and the walk shape: L vertices per walk, window W (pairs of walk
    positions less than W apart), Bw walks per batch (the sample order interleaves a
    batch's walks)."""

    def __init__(self, tables: "Tables", L: int = 100, W: int = 2, Bw: int = 1 << 17):
        t = tables
        self.t, self.L, self.W, self.Bw = t, int(L), int(W), int(Bw)
        self.off = np.zeros(t.n + 1, dtype=np.int64)
        self.nbr = np.zeros(2 * t.m, dtype=np.int32)
        self.wt = np.zeros(2 * t.m, dtype=np.float64)
        if lib().or_walk_csr(t.n, t.m, _p(t.src), _p(t.dst), _p(t.w), _p(self.off), _p(self.nbr),
                             _p(self.wt)) != 0:
            raise ValueError("or_walk_csr rejected its arguments")
        self.thr = np.zeros(2 * t.m, dtype=np.uint64)
        self.alias = np.zeros(2 * t.m, dtype=np.int32)
        lib().or_walk_alias(t.n, _p(self.off), _p(self.wt), _p(self.thr), _p(self.alias))

    @property
    def pairs_per_walk(self) -> int:
        return sum(self.L - dl for dl in range(1, self.W))

    def _args(self):
        t = self.t
        return (t.n, t.m, _p(t.src), _p(t.dst), _p(t.ethr), _p(t.ealias), _p(self.off), _p(self.nbr),
                _p(self.thr), _p(self.alias))

    def pairs(self, seed: int, graph_id: int, first: int, count: int):
        """(u, v) of samples [first, first + count)."""
        u = np.zeros(count, dtype=np.int32)
        v = np.zeros(count, dtype=np.int32)
        if lib().or_walk_pairs(*self._args(), seed, graph_id, self.L, self.W, self.Bw, first, count,
                               _p(u), _p(v)) != 0:
            raise ValueError("or_walk_pairs rejected its arguments")
        return u, v

    def pool(self, seed: int, graph_id: int, R: int, first: int = 0, count: int = 0):
        """The pair pool of R collected walk pairs (Sec. IV-C, Augmented-Pair): returns
        (pool_u, pool_v, u, v), the collected pairs and the positive pairs samples
        [first, first + count) draw from them."""
        pu = np.zeros(R, dtype=np.int32)
        pv = np.zeros(R, dtype=np.int32)
        u = np.zeros(max(count, 1), dtype=np.int32)
        v = np.zeros(max(count, 1), dtype=np.int32)
        if lib().or_pool_pairs(*self._args(), seed, graph_id, self.L, self.W, self.Bw, R, _p(pu), _p(pv),
                               first, count, _p(u), _p(v)) != 0:
            raise ValueError("or_pool_pairs rejected its arguments")
        return pu, pv, u[:count], v[:count]

    def walks(self, seed: int, graph_id: int, k0: int, nwalks: int) -> np.ndarray:
        """Vertices of walks k0 .. k0 + nwalks - 1, [nwalks, L]."""
        out = np.zeros((nwalks, self.L), dtype=np.int32)
        if lib().or_walk_vertices(*self._args(), seed, graph_id, self.L, k0, nwalks, _p(out)) != 0:
            raise ValueError("or_walk_vertices rejected its arguments")
        return out


def pool_size(T: int) -> int:
    """Pairs a pool collects for a run of T samples: the least R >= 2 with
    R (R - 1) / 2 >= T (about sqrt(2 T), Sec. IV-C)."""
    return int(lib().or_pool_size(T))


def sample(t: Tables, seed: int, graph_id: int, K: int, first: int, count: int):
    """Sampled tuples (u, v, neg[count, K]) for sample indices [first, first+count)."""
    u = np.zeros(count, dtype=np.int32)
    v = np.zeros(count, dtype=np.int32)
    neg = np.zeros(count * max(K, 1), dtype=np.int32)
    lib().or_sample(t.n, t.m, _p(t.src), _p(t.dst), _p(t.ethr), _p(t.ealias), _p(t.nthr),
                    _p(t.nalias), seed, graph_id, K, first, count, _p(u), _p(v), _p(neg))
    return u, v, neg[: count * K].reshape(count, K)


def sample_negatives(n: int, nthr, nalias, seed: int, graph_id: int, K: int, first: int,
                     count: int) -> np.ndarray:
    """Negatives (count x K) of sample indices [first, first+count) from a negative table
    alone: slot j of sample s draws from Block(key = (seed, graph_id), ctr = (s, j, 0, 0))
    exactly as ``sample`` does (Algorithm 1, v- ~ q of Eq. (1))."""
    nthr = _c(nthr, np.uint64)
    nalias = _c(nalias, np.int32)
    assert nthr.size == n and nalias.size == n
    neg = np.zeros(count * max(K, 1), dtype=np.int32)
    lib().or_sample_negatives(n, _p(nthr), _p(nalias), seed, graph_id, K, first, count, _p(neg))
    return neg[: count * K].reshape(count, K)


def init_table(t: int, rows: int, d: int, seed: int, graph_id: int) -> np.ndarray:
    """Initial table t (0 = U, 1 = C, 2 = U1): uniform on [-0.5/d, 0.5/d), float32."""
    out = np.zeros((rows, d), dtype=np.float32)
    lib().or_init_table(_p(out), t, rows, d, seed, graph_id)
    return out


def bf16_rne(x) -> np.ndarray:
    """Nearest bfloat16 (ties to even) of the binary32 rounding of each value (float64 out)."""
    y = _c(x, np.float64).copy()
    lib().or_bf16_rne(_p(y), y.size)
    return y


def sr_bf16(x: float, bits: int) -> float:
    """Stochastic rounding of x to bfloat16 with 16 given random bits (after rounding x to
    binary32): the value the bfloat16 storage mode writes."""
    return float(lib().or_sr_bf16(float(x), int(bits)))


class Model:
    """Embedding tables plus the hyper-parameters of Algorithm 1.  ``storage``: "binary64"
    (the default), or "bf16" -- tables held as bfloat16 values (initial values rounded to
    nearest, every written value stochastically rounded; SEQ mode only), the precision
    extension's storage.  ``sr_stream`` selects one of independent streams of rounding bits
    (bfloat16 storage only)."""

    def __init__(self, tables: Tables, d: int, K: int, orders: int, T: int, seed: int,
                 graph_id: int = 0, eta0: float = 0.025, lam: float = 0.0, alpha: float = 1.0,
                 storage: str = "binary64", sr_stream: int = 0):
        if storage not in ("binary64", "bf16"):
            raise ValueError(storage)
        self.t, self.d, self.K, self.orders, self.T = tables, d, K, orders, T
        self.seed, self.graph_id = seed, graph_id
        self.eta0, self.lam, self.alpha = eta0, lam, alpha
        self.storage = storage
        self.sr_stream = int(sr_stream)
        n = tables.n
        self.U = self.C = self.U1 = None
        if orders & 2:
            self.U = init_table(0, n, d, seed, graph_id).astype(np.float64)
            self.C = init_table(1, n, d, seed, graph_id).astype(np.float64)
        if orders & 1:
            self.U1 = init_table(2, n, d, seed, graph_id).astype(np.float64)
        if storage == "bf16":
            for X in (self.U, self.C, self.U1):
                if X is not None:
                    lib().or_bf16_rne(_p(X), X.size)

    def train(self, first: int, count: int, mode: str = "seq", batch: int = 0,
              walks: Optional["WalkGraph"] = None, pool: int = 0):
        """SEQ (each sample applied at once) or SNAPSHOT (Eq. (4) per batch).  ``walks``:
        positive pairs from that random-walk source instead of arc draws; with ``pool`` = R
        > 0, from the pair pool of R pairs collected from it (Sec. IV-C, Augmented-Pair)."""
        t = self.t
        if pool:
            if walks is None:
                raise ValueError("a pair pool is collected from a walk source")
            if self.storage == "bf16" and mode != "seq":
                raise ValueError("bfloat16 storage is modelled in SEQ mode only")
            wg = walks
            rc = lib().or_train_pool(_p(t.src), _p(t.dst), t.n, t.m, _p(t.ethr), _p(t.ealias),
                                     _p(t.nthr), _p(t.nalias), _p(wg.off), _p(wg.nbr), _p(wg.thr),
                                     _p(wg.alias), wg.L, wg.W, wg.Bw, int(pool), self.seed, self.graph_id,
                                     self.d, self.K, self.orders, self.eta0, self.lam, self.alpha, self.T,
                                     _p(self.U), _p(self.C), _p(self.U1), first, count,
                                     0 if mode == "seq" else 1, batch,
                                     self.sr_stream if self.storage == "bf16" else -1)
            if rc != 0:
                raise ValueError("or_train_pool rejected its arguments")
            return
        if walks is not None and self.storage == "bf16":
            if mode != "seq":
                raise ValueError("bfloat16 storage is modelled in SEQ mode only")
            wg = walks
            rc = lib().or_train_bf16_walk(_p(t.src), _p(t.dst), t.n, t.m, _p(t.ethr), _p(t.ealias),
                                          _p(t.nthr), _p(t.nalias), _p(wg.off), _p(wg.nbr), _p(wg.thr),
                                          _p(wg.alias), wg.L, wg.W, wg.Bw, self.seed, self.graph_id,
                                          self.d, self.K, self.orders, self.eta0, self.lam, self.alpha,
                                          self.T, _p(self.U), _p(self.C), _p(self.U1), first, count,
                                          self.sr_stream)
            if rc != 0:
                raise ValueError("or_train_bf16_walk rejected its arguments")
            return
        if walks is not None:
            wg = walks
            rc = lib().or_train_walk(_p(t.src), _p(t.dst), t.n, t.m, _p(t.ethr), _p(t.ealias),
                                     _p(t.nthr), _p(t.nalias), _p(wg.off), _p(wg.nbr), _p(wg.thr),
                                     _p(wg.alias), wg.L, wg.W, wg.Bw, self.seed, self.graph_id, self.d,
                                     self.K, self.orders, self.eta0, self.lam, self.alpha, self.T,
                                     _p(self.U), _p(self.C), _p(self.U1), first, count,
                                     0 if mode == "seq" else 1, batch)
            if rc != 0:
                raise ValueError("or_train_walk rejected its arguments")
            return
        if self.storage == "bf16":
            if mode != "seq":
                raise ValueError("bfloat16 storage is modelled in SEQ mode only")
            rc = lib().or_train_bf16(_p(t.src), _p(t.dst), t.n, t.m, _p(t.ethr), _p(t.ealias),
                                     _p(t.nthr), _p(t.nalias), self.seed, self.graph_id, self.d,
                                     self.K, self.orders, self.eta0, self.lam, self.alpha, self.T,
                                     _p(self.U), _p(self.C), _p(self.U1), first, count,
                                     self.sr_stream)
            if rc != 0:
                raise ValueError("or_train_bf16 rejected its arguments")
            return
        rc = lib().or_train(_p(t.src), _p(t.dst), t.n, t.m, _p(t.ethr), _p(t.ealias),
                            _p(t.nthr), _p(t.nalias), self.seed, self.graph_id, self.d, self.K,
                            self.orders, self.eta0, self.lam, self.alpha, self.T, _p(self.U),
                            _p(self.C), _p(self.U1), first, count,
                            0 if mode == "seq" else 1, batch)
        if rc != 0:
            raise ValueError("or_train rejected its arguments")

    def scores(self, u, v, order: int) -> np.ndarray:
        """Link score: U[u].C[v] (order 2) or U1[u].U1[v] (order 1), binary64."""
        A, B = (self.U, self.C) if order == 2 else (self.U1, self.U1)
        return pair_scores(A, B, u, v)


def pair_scores(A, B, u, v) -> np.ndarray:
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    u = _c(u, np.int32)
    v = _c(v, np.int32)
    out = np.zeros(u.size, dtype=np.float64)
    lib().or_pair_scores(_p(A), _p(B), A.shape[1], _p(u), _p(v), u.size, _p(out))
    return out


def train_hogwild_f32(tables: Tables, U, C, U1, d, K, orders, T, seed, graph_id, first, count,
                      nthreads, eta0=0.025, lam=0.0, alpha=1.0):
    """Binary32 lock-free timing mode on ``nthreads`` OpenMP threads (tables updated in place)."""
    t = tables
    rc = lib().or_train_hogwild_f32(_p(t.src), _p(t.dst), t.n, t.m, _p(t.ethr), _p(t.ealias),
                                    _p(t.nthr), _p(t.nalias), seed, graph_id, d, K, orders,
                                    eta0, lam, alpha, T, _p(U), _p(C), _p(U1), first, count,
                                    nthreads)
    if rc != 0:
        raise ValueError("or_train_hogwild_f32 rejected its arguments")


def max_threads() -> int:
    return int(lib().or_max_threads())


def auc(pos, neg) -> float:
    """Mann-Whitney AUC of positive vs negative scores, ties counted one half."""
    p = _c(pos, np.float64)
    q = _c(neg, np.float64)
    return float(lib().or_auc(_p(p), p.size, _p(q), q.size))
