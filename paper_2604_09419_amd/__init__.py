"""linehip: LINE-style edge-sampled SGD on AMD Instinct MI355X (gfx950).

The method (NOMAD, arXiv 2604.09419, Sec. IV "Methods"): positive pairs are arcs drawn from the
weight-normalised edge distribution (Algorithm 3, root-edge selection), K negatives per
pair are drawn from q(v) ~ out-degree^0.75 (Eq. (1)), and the vertex and context
embedding tables receive the SGD updates of Algorithm 1 / Eqs. (2)-(3); a deterministic
SNAPSHOT mode applies per-row batch sums as in Eq. (4).

This package is a thin layer over the C ABI of ``liblinehip.so`` (``_lib``, same names as
include/linehip.h).  ``Trainer`` and ``BatchTrainer`` add only device-memory management
with torch tensors and a torch stream; every step of the method runs in the HIP kernels.
"""
from __future__ import annotations

from typing import Optional, Sequence

from . import _lib
from ._lib import (  # noqa: F401
    LH_ALIAS_EDGE, LH_ALIAS_NEG, LH_BF16, LH_FP32, LH_HOGWILD, LH_ORDER1, LH_ORDER2, LH_ORDER12,
    LH_SNAPSHOT, LH_TABLE_C, LH_TABLE_U, LH_TABLE_U1, LhError, lib, make_params,
)

__all__ = ["Trainer", "BatchTrainer", "LhError", "lib", "make_params"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("linehip needs a HIP GPU (torch.cuda.is_available() is False)")
    return torch


class Trainer:
    """One graph's tables, alias tables and workspace on one GPU.

    ``src``, ``dst`` (int32) and ``w`` (float32) may be numpy arrays or torch tensors.
    ``orders``: 1 (first), 2 (second) or 3 (both).  ``dtype``: "fp32" or "bf16".
    ``mode``: "hogwild" or "snapshot" (then ``batch`` samples per snapshot).
    ``hot_shadow`` (bfloat16 Hogwild): hot rows accumulate in a binary32 shadow for each
    launch instead of taking stochastically rounded packed bfloat16 atomics.
    """

    def __init__(self, n: int, src, dst, w, d: int, K: int = 5, orders: int = 2, dtype: str = "fp32",
                 eta0: float = 0.025, lam: float = 0.0, alpha_neg: float = 1.0, seed: int = 1,
                 total_samples: int = 1, mode: str = "hogwild", batch: int = 0, graph_id: int = 0,
                 hot_rate: float = 0.75, max_conflicts: float = 0.25, hot_shadow: bool = False,
                 device: int = 0, stream=None, build: bool = True, init: bool = True):
        torch = _torch()
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.n, self.d, self.K, self.orders = int(n), int(d), int(K), int(orders)
        self.dtype = dtype
        self.T = int(total_samples)
        self.params = make_params(d=d, K=K, orders=orders, dtype=LH_FP32 if dtype == "fp32" else LH_BF16,
                                  eta0=eta0, lam=lam, alpha_neg=alpha_neg, seed=seed, total_samples=total_samples,
                                  mode=LH_HOGWILD if mode == "hogwild" else LH_SNAPSHOT, graph_id=graph_id,
                                  batch=batch, hot_rate=hot_rate, max_conflicts=max_conflicts,
                                  hot_shadow=hot_shadow)
        self.h = _lib.lh_create(self.params, device)
        tdt = torch.float32 if dtype == "fp32" else torch.bfloat16
        # Inputs given as GPU tensors may still be in the making on the caller's stream.
        self._after_caller()
        with torch.cuda.stream(self.stream):
            self.src = torch.as_tensor(src, dtype=torch.int32).to(self.device).contiguous()
            self.dst = torch.as_tensor(dst, dtype=torch.int32).to(self.device).contiguous()
            self.w = torch.as_tensor(w, dtype=torch.float32).to(self.device).contiguous()
            self.m = int(self.src.numel())
            persist, self.scratch_bytes = _lib.lh_workspace_size(self.params, self.n, self.m)
            self.ws = torch.empty(persist + 256, dtype=torch.uint8, device=self.device)
            self.tables = [None, None, None]
            if orders & 2:
                self.tables[LH_TABLE_U] = torch.empty((self.n, d), dtype=tdt, device=self.device)
                self.tables[LH_TABLE_C] = torch.empty((self.n, d), dtype=tdt, device=self.device)
            if orders & 1:
                self.tables[LH_TABLE_U1] = torch.empty((self.n, d), dtype=tdt, device=self.device)
        ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        _lib.lh_bind(self.h, ws_ptr, persist, [t.data_ptr() if t is not None else 0 for t in self.tables],
                     self.stream.cuda_stream)
        _lib.lh_set_graph(self.h, self.n, self.m, self.src.data_ptr(), self.dst.data_ptr(), self.w.data_ptr())
        if build:
            self.build_alias()
        if init:
            self.init_embeddings()

    def _after_caller(self):
        """Order this trainer's stream after the caller's current stream (work the caller
        queued there, such as producing an input tensor, finishes first)."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    # -- the C calls ---------------------------------------------------------------------
    def build_alias(self):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            scratch = torch.empty(self.scratch_bytes + 256, dtype=torch.uint8, device=self.device)
        _lib.lh_build_alias(self.h, (scratch.data_ptr() + 255) // 256 * 256, self.scratch_bytes)
        del scratch  # lh_build_alias synchronised the stream

    def init_embeddings(self):
        _lib.lh_init_embeddings(self.h)

    def build_walks(self, walk_length: int = 100, window: int = 2, walks_per_batch: int = 1024):
        """Switch the positive pairs to random walks (Sec. IV-B, Algorithms 2-3): builds the
        walk graph's rows and per-row alias tables; later training and sampling calls take
        their pairs from the walks."""
        torch = self.torch
        persist, scratch_bytes = _lib.lh_walk_size(self.n, self.m, walk_length, window, walks_per_batch)
        with torch.cuda.stream(self.stream):
            self.walk_mem = torch.empty(persist + 256, dtype=torch.uint8, device=self.device)
            scratch = torch.empty(scratch_bytes + 256, dtype=torch.uint8, device=self.device)
        _lib.lh_walk_build(self.h, walk_length, window, walks_per_batch, (self.walk_mem.data_ptr() + 255) // 256 * 256,
                           persist, (scratch.data_ptr() + 255) // 256 * 256, scratch_bytes)
        del scratch  # lh_walk_build synchronised the stream
        self.walk_shape = (int(walk_length), int(window), int(walks_per_batch))

    def walk_pairs(self, first: int, count: int):
        """(u, v) of samples [first, first + count) from the walks, as training takes them."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            u = torch.empty(max(count, 1), dtype=torch.int32, device=self.device)
            v = torch.empty(max(count, 1), dtype=torch.int32, device=self.device)
        _lib.lh_walk_pairs(self.h, first, count, u.data_ptr(), v.data_ptr())
        self.stream.synchronize()
        return u[:count], v[:count]

    def walk_export(self):
        """(row offsets int64 [n + 1], thr uint64 [2m], keep int32 [2m], alias int32 [2m]) of
        the walk rows as numpy arrays: entry i keeps its head keep[i] when the draw's
        threshold word is below thr[i], else yields alias[i]."""
        import numpy as np
        torch = self.torch
        E = 2 * self.m
        with torch.cuda.stream(self.stream):
            off = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
            thr = torch.empty(E, dtype=torch.int64, device=self.device)
            keep = torch.empty(E, dtype=torch.int32, device=self.device)
            al = torch.empty(E, dtype=torch.int32, device=self.device)
        _lib.lh_walk_export(self.h, off.data_ptr(), thr.data_ptr(), keep.data_ptr(), al.data_ptr())
        return off.cpu().numpy(), thr.cpu().numpy().view(np.uint64), keep.cpu().numpy(), al.cpu().numpy()

    def detach_walks(self):
        _lib.lh_walk_detach(self.h)

    def build_pool(self, pairs: int = 0):
        """Draw the positive pairs from a pool of walk pairs collected up front (Sec. IV-C,
        Augmented-Pair): ``pairs`` = R collected pairs, by default the library's size for
        this handle's total_samples (about sqrt(2 T)).  Needs build_walks first."""
        R = int(pairs) if pairs else _lib.lh_walk_pool_size(self.T)
        _lib.lh_walk_pool(self.h, R)
        self.pool_pairs = R
        return R

    def drop_pool(self):
        """Back to the walk pairs."""
        _lib.lh_walk_pool(self.h, 0)
        self.pool_pairs = 0

    def import_alias(self, which: int, thr, alias):
        torch = self.torch
        self._after_caller()
        with torch.cuda.stream(self.stream):
            t = torch.as_tensor(thr.view("int64") if hasattr(thr, "view") and not torch.is_tensor(thr) else thr)
            t = t.to(self.device, torch.int64).contiguous()
            a = torch.as_tensor(alias, dtype=torch.int32).to(self.device).contiguous()
        _lib.lh_import_alias(self.h, which, t.data_ptr(), a.data_ptr())
        self.stream.synchronize()

    def export_alias(self, which: int):
        """(thr as uint64 numpy array, alias as int32 numpy array)."""
        import numpy as np
        torch = self.torch
        N = self.m if which == LH_ALIAS_EDGE else self.n
        with torch.cuda.stream(self.stream):
            t = torch.empty(N, dtype=torch.int64, device=self.device)
            a = torch.empty(N, dtype=torch.int32, device=self.device)
        _lib.lh_export_alias(self.h, which, t.data_ptr(), a.data_ptr())
        return t.cpu().numpy().view(np.uint64), a.cpu().numpy()

    def sample(self, first: int, count: int):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            u = torch.empty(count, dtype=torch.int32, device=self.device)
            v = torch.empty(count, dtype=torch.int32, device=self.device)
            neg = torch.empty(max(count * self.K, 1), dtype=torch.int32, device=self.device)
        _lib.lh_sample(self.h, first, count, u.data_ptr(), v.data_ptr(), neg.data_ptr())
        self.stream.synchronize()
        return u, v, neg[: count * self.K].view(count, self.K)

    def train_steps(self, first: int, count: int):
        _lib.lh_train_steps(self.h, first, count)

    def last_train_ms(self) -> float:
        return _lib.lh_last_train_ms(self.h)

    def tune(self, probe: int, cache_path: Optional[str] = None):
        _lib.lh_tune(self.h, probe, cache_path)

    def kernel_config(self):
        return _lib.lh_kernel_config(self.h)

    def set_kernel_config(self, lanes_per_sample: int, units_per_lane: int, blocks_per_cu: int):
        _lib.lh_set_kernel_config(self.h, lanes_per_sample, units_per_lane, blocks_per_cu)

    def read(self, table: int, row0: int = 0, rows: Optional[int] = None):
        """Rows of table ``table`` as a float32 tensor on the GPU (bfloat16 widened)."""
        torch = self.torch
        rows = self.n - row0 if rows is None else rows
        with torch.cuda.stream(self.stream):
            out = torch.empty((rows, self.d), dtype=torch.float32, device=self.device)
        _lib.lh_read_embeddings(self.h, table, row0, rows, out.data_ptr())
        self.stream.synchronize()
        return out

    def write(self, table: int, x, row0: int = 0):
        torch = self.torch
        self._after_caller()
        with torch.cuda.stream(self.stream):
            xt = torch.as_tensor(x, dtype=torch.float32).to(self.device).contiguous()
        _lib.lh_write_embeddings(self.h, table, row0, xt.shape[0], xt.data_ptr())
        self.stream.synchronize()

    def check(self):
        _lib.lh_check(self.h)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "h", None):
            _lib.lh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchTrainer:
    """Many second-order Hogwild ``Trainer``s (same stream, dtype) trained in one persistent
    launch; ``capture()`` records it into a hipGraph, ``launch()`` replays it."""

    def __init__(self, trainers: Sequence[Trainer]):
        self.trainers = list(trainers)
        self.b = _lib.lh_batch_create([t.h for t in self.trainers])

    def tune(self, cache_path: Optional[str] = None):
        _lib.lh_batch_tune(self.b, cache_path)

    def capture(self):
        _lib.lh_batch_capture(self.b)

    def launch(self, stream=None):
        """Replay the captured launch on ``stream`` (a torch stream; None: the trainers'
        stream)."""
        _lib.lh_batch_launch(self.b, stream.cuda_stream if stream is not None else 0)

    def run(self, stream=None):
        _lib.lh_batch_run(self.b, stream.cuda_stream if stream is not None else 0)

    def last_ms(self) -> float:
        return _lib.lh_batch_last_ms(self.b)

    def done(self):
        return _lib.lh_batch_done(self.b, len(self.trainers))

    def close(self):
        if getattr(self, "b", None):
            _lib.lh_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
