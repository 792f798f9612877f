"""ctypes binding of liblinehip.so: the C ABI of include/linehip.h with the same names.

Argument marshalling only: every step of the method runs in the HIP kernels of the
library.  Loading fails loudly when the built library is missing; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "liblinehip.so")

LH_OK = 0
STATUS_NAMES = {
    0: "LH_OK", 1: "LH_ERR_INVALID_ARG", 2: "LH_ERR_OUT_OF_RANGE", 3: "LH_ERR_ZERO_WEIGHT",
    4: "LH_ERR_WORKSPACE_TOO_SMALL", 5: "LH_ERR_NOT_BUILT", 6: "LH_ERR_UNSUPPORTED",
    7: "LH_ERR_NO_DEVICE", 8: "LH_ERR_HIP",
}
LH_FP32, LH_BF16 = 0, 1
LH_HOGWILD, LH_SNAPSHOT = 0, 1
LH_ORDER1, LH_ORDER2, LH_ORDER12 = 1, 2, 3
LH_TABLE_U, LH_TABLE_C, LH_TABLE_U1 = 0, 1, 2
LH_ALIAS_EDGE, LH_ALIAS_NEG = 0, 1


class lh_params(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("orders", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("eta0", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("alpha_neg", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("total_samples", ctypes.c_uint64),
        ("mode", ctypes.c_int32),
        ("graph_id", ctypes.c_int32),
        ("batch", ctypes.c_int64),
        ("hot_rate", ctypes.c_double),
        ("max_conflicts", ctypes.c_double),
        ("hot_shadow", ctypes.c_int32),
    ]


class LhError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {name}" + (f" ({detail})" if detail else ""))


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblinehip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise ImportError(f"{SO_PATH} is missing: build it with `python -m paper_2604_09419_amd.build`")
    L = ctypes.CDLL(SO_PATH)
    P, S = ctypes.c_void_p, ctypes.c_int
    i64, u64, sz = ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "lh_create": [PP, ctypes.POINTER(lh_params), S],
        "lh_workspace_size": [ctypes.POINTER(lh_params), i64, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "lh_bind": [P, P, sz, ctypes.POINTER(ctypes.c_void_p * 3), P],
        "lh_set_graph": [P, i64, i64, P, P, P],
        "lh_build_alias": [P, P, sz],
        "lh_build_alias_noalloc": [P],
        "lh_import_alias": [P, S, P, P],
        "lh_export_alias": [P, S, P, P],
        "lh_init_embeddings": [P],
        "lh_sample": [P, u64, u64, P, P, P],
        "lh_train_steps": [P, u64, u64],
        "lh_tune": [P, u64, ctypes.c_char_p],
        "lh_read_embeddings": [P, S, i64, i64, P],
        "lh_write_embeddings": [P, S, i64, i64, P],
        "lh_check": [P],
        "lh_last_train_ms": [P, ctypes.POINTER(ctypes.c_double)],
        "lh_kernel_config": [P, ctypes.POINTER(ctypes.c_int32 * 3)],
        "lh_set_kernel_config": [P, ctypes.POINTER(ctypes.c_int32 * 3)],
        "lh_destroy": [P],
        "lh_batch_create": [PP, S, ctypes.POINTER(ctypes.c_void_p)],
        "lh_batch_tune": [P, ctypes.c_char_p],
        "lh_batch_capture": [P],
        "lh_batch_launch": [P, P],
        "lh_batch_run": [P, P],
        "lh_batch_last_ms": [P, ctypes.POINTER(ctypes.c_double)],
        "lh_batch_config": [P, ctypes.POINTER(ctypes.c_int64 * 3)],
        "lh_batch_done": [P, P],
        "lh_batch_destroy": [P],
        "lh_walk_size": [i64, i64, ctypes.c_int32, ctypes.c_int32, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "lh_walk_build": [P, ctypes.c_int32, ctypes.c_int32, i64, P, sz, P, sz],
        "lh_walk_pairs": [P, u64, u64, P, P],
        "lh_walk_export": [P, P, P, P, P],
        "lh_walk_detach": [P],
        "lh_walk_pool_size": [u64, ctypes.POINTER(u64)],
        "lh_walk_pool": [P, u64],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = S
    L.lh_status_string.argtypes = [S]
    L.lh_status_string.restype = ctypes.c_char_p
    L.lh_last_error.argtypes = [P]
    L.lh_last_error.restype = ctypes.c_char_p
    L.lh_abi_symbol_count.argtypes = []
    L.lh_abi_symbol_count.restype = S
    L.lh_abi_symbol_name.argtypes = [S]
    L.lh_abi_symbol_name.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int, where: str, handle=None) -> None:
    if status != LH_OK:
        detail = ""
        if handle:
            raw = lib().lh_last_error(handle)
            detail = raw.decode() if raw else ""
        raise LhError(status, where, detail)


def make_params(d: int, K: int = 5, orders: int = LH_ORDER2, dtype: int = LH_FP32, eta0: float = 0.025,
                lam: float = 0.0, alpha_neg: float = 1.0, seed: int = 1, total_samples: int = 1,
                mode: int = LH_HOGWILD, graph_id: int = 0, batch: int = 0,
                hot_rate: float = 0.75, max_conflicts: float = 0.25, hot_shadow: bool = False) -> lh_params:
    return lh_params(d, K, orders, dtype, eta0, lam, alpha_neg, seed, total_samples, mode, graph_id, batch,
                     hot_rate, max_conflicts, int(bool(hot_shadow)))


# ---- the C entry points, same names -----------------------------------------------------
def lh_create(p: lh_params, device: int = 0):
    h = ctypes.c_void_p()
    check(lib().lh_create(ctypes.byref(h), ctypes.byref(p), device), "lh_create")
    return h


def lh_workspace_size(p: lh_params, n: int, m: int):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().lh_workspace_size(ctypes.byref(p), n, m, ctypes.byref(a), ctypes.byref(b)), "lh_workspace_size")
    return a.value, b.value


def lh_bind(h, workspace_ptr: int, nbytes: int, tables, stream: int):
    arr = (ctypes.c_void_p * 3)(*[t or None for t in tables])
    check(lib().lh_bind(h, workspace_ptr, nbytes, ctypes.byref(arr), stream or None), "lh_bind", h)


def lh_set_graph(h, n: int, m: int, src_ptr: int, dst_ptr: int, w_ptr: int):
    check(lib().lh_set_graph(h, n, m, src_ptr or None, dst_ptr or None, w_ptr or None), "lh_set_graph", h)


def lh_build_alias(h, scratch_ptr: int, nbytes: int):
    check(lib().lh_build_alias(h, scratch_ptr or None, nbytes), "lh_build_alias", h)


def lh_build_alias_noalloc(h):
    check(lib().lh_build_alias_noalloc(h), "lh_build_alias_noalloc", h)


def lh_import_alias(h, which: int, thr_ptr: int, alias_ptr: int):
    check(lib().lh_import_alias(h, which, thr_ptr or None, alias_ptr or None), "lh_import_alias", h)


def lh_export_alias(h, which: int, thr_ptr: int, alias_ptr: int):
    check(lib().lh_export_alias(h, which, thr_ptr or None, alias_ptr or None), "lh_export_alias", h)


def lh_init_embeddings(h):
    check(lib().lh_init_embeddings(h), "lh_init_embeddings", h)


def lh_sample(h, first: int, count: int, u_ptr: int, v_ptr: int, neg_ptr: int):
    check(lib().lh_sample(h, first, count, u_ptr or None, v_ptr or None, neg_ptr or None), "lh_sample", h)


def lh_train_steps(h, first: int, count: int):
    check(lib().lh_train_steps(h, first, count), "lh_train_steps", h)


def lh_tune(h, probe: int, cache_path=None):
    check(lib().lh_tune(h, probe, cache_path.encode() if cache_path else None), "lh_tune", h)


def lh_read_embeddings(h, table: int, row0: int, rows: int, out_ptr: int):
    check(lib().lh_read_embeddings(h, table, row0, rows, out_ptr or None), "lh_read_embeddings", h)


def lh_write_embeddings(h, table: int, row0: int, rows: int, in_ptr: int):
    check(lib().lh_write_embeddings(h, table, row0, rows, in_ptr or None), "lh_write_embeddings", h)


def lh_check(h):
    check(lib().lh_check(h), "lh_check", h)


def lh_last_train_ms(h) -> float:
    ms = ctypes.c_double()
    check(lib().lh_last_train_ms(h, ctypes.byref(ms)), "lh_last_train_ms", h)
    return ms.value


def lh_kernel_config(h):
    out = (ctypes.c_int32 * 3)()
    check(lib().lh_kernel_config(h, ctypes.byref(out)), "lh_kernel_config", h)
    return {"lanes_per_sample": out[0], "units_per_lane": out[1], "blocks_per_cu": out[2]}


def lh_set_kernel_config(h, lanes_per_sample: int, units_per_lane: int, blocks_per_cu: int):
    arr = (ctypes.c_int32 * 3)(lanes_per_sample, units_per_lane, blocks_per_cu)
    check(lib().lh_set_kernel_config(h, ctypes.byref(arr)), "lh_set_kernel_config", h)


def lh_destroy(h):
    check(lib().lh_destroy(h), "lh_destroy")


def lh_batch_create(handles):
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    b = ctypes.c_void_p()
    check(lib().lh_batch_create(ctypes.byref(b), len(handles), arr), "lh_batch_create")
    return b


def lh_batch_tune(b, cache_path=None):
    check(lib().lh_batch_tune(b, cache_path.encode() if cache_path else None), "lh_batch_tune")


def lh_batch_capture(b):
    check(lib().lh_batch_capture(b), "lh_batch_capture")


def lh_batch_launch(b, stream: int = 0):
    check(lib().lh_batch_launch(b, stream or None), "lh_batch_launch")


def lh_batch_run(b, stream: int = 0):
    check(lib().lh_batch_run(b, stream or None), "lh_batch_run")


def lh_batch_last_ms(b) -> float:
    ms = ctypes.c_double()
    check(lib().lh_batch_last_ms(b, ctypes.byref(ms)), "lh_batch_last_ms")
    return ms.value


def lh_batch_config(b):
    out = (ctypes.c_int64 * 3)()
    check(lib().lh_batch_config(b, ctypes.byref(out)), "lh_batch_config")
    return {"variant": out[0], "blocks_per_cu": out[1], "item_samples": out[2]}


def lh_batch_done(b, G: int):
    out = (ctypes.c_uint64 * G)()
    check(lib().lh_batch_done(b, out), "lh_batch_done")
    return list(out)


def lh_batch_destroy(b):
    check(lib().lh_batch_destroy(b), "lh_batch_destroy")


def lh_walk_size(n: int, m: int, walk_length: int, window: int, walks_per_batch: int):
    persist, scratch = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().lh_walk_size(n, m, walk_length, window, walks_per_batch, ctypes.byref(persist),
                             ctypes.byref(scratch)), "lh_walk_size")
    return persist.value, scratch.value


def lh_walk_build(h, walk_length: int, window: int, walks_per_batch: int, persist_ptr: int, persist_bytes: int,
                  scratch_ptr: int, scratch_bytes: int):
    check(lib().lh_walk_build(h, walk_length, window, walks_per_batch, persist_ptr or None, persist_bytes,
                              scratch_ptr or None, scratch_bytes), "lh_walk_build", h)


def lh_walk_pairs(h, first: int, count: int, u_ptr: int, v_ptr: int):
    check(lib().lh_walk_pairs(h, first, count, u_ptr or None, v_ptr or None), "lh_walk_pairs", h)


def lh_walk_export(h, off_ptr: int, thr_ptr: int, keep_ptr: int, alias_ptr: int):
    check(lib().lh_walk_export(h, off_ptr or None, thr_ptr or None, keep_ptr or None, alias_ptr or None),
          "lh_walk_export", h)


def lh_walk_detach(h):
    check(lib().lh_walk_detach(h), "lh_walk_detach", h)


def lh_walk_pool_size(total_samples: int) -> int:
    pairs = ctypes.c_uint64()
    check(lib().lh_walk_pool_size(total_samples, ctypes.byref(pairs)), "lh_walk_pool_size")
    return pairs.value


def lh_walk_pool(h, pairs: int):
    check(lib().lh_walk_pool(h, pairs), "lh_walk_pool", h)


def lh_abi_symbols():
    L = lib()
    return [L.lh_abi_symbol_name(i).decode() for i in range(L.lh_abi_symbol_count())]
