"""ctypes binding of libials (argument marshalling only).

Every function here has the name of the C entry point it calls and does
nothing but convert arguments; all of the work runs in the HIP kernels of
libials.so.  PyTorch supplies device memory and streams.  If the library has
not been built, loading fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# IALS_LIB selects another build of the same sources (the host sanitizer test uses it)
LIB_PATH = os.environ.get("IALS_LIB") or os.path.join(_PKG, "libials.so")

IALS_OK = 0
IALS_E_INVALID = -1
IALS_E_NOMEM = -2
IALS_E_HIP = -3
IALS_E_NOT_SPD = -4
IALS_E_BUSY = -5
IALS_E_STATE = -6
IALS_SOLVER_BLOCK = 0
IALS_SOLVER_IALS = 1
IALS_SOLVER_ICD = 2

IALS_SIDE_USER = 0
IALS_SIDE_ITEM = 1
IALS_MAT_W = 0
IALS_MAT_H = 1
IALS_MEM_HOST = 0
IALS_MEM_DEVICE = 1
IALS_PREC_FP32 = 0
IALS_PREC_BF16 = 1
IALS_FLAG_GRAPH = 1
IALS_FLAG_DEAL_QUEUE = 2
IALS_FLAG_DEAL_STATIC = 4

_STATUS_NAMES = {0: "IALS_OK", -1: "IALS_E_INVALID", -2: "IALS_E_NOMEM", -3: "IALS_E_HIP",
                 -4: "IALS_E_NOT_SPD", -5: "IALS_E_BUSY", -6: "IALS_E_STATE"}


class ials_config(C.Structure):
    _fields_ = [("num_users", C.c_int32), ("num_items", C.c_int32), ("dim", C.c_int32),
                ("block", C.c_int32), ("alpha0", C.c_float), ("lambda_", C.c_float),
                ("precision", C.c_int32), ("chol_fallback_ratio", C.c_float), ("flags", C.c_uint32),
                ("seg_len", C.c_uint32), ("hbm_budget", C.c_uint64), ("gram_split", C.c_uint32),
                ("reserved", C.c_uint32)]


class ials_coo(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("user", C.c_void_p), ("item", C.c_void_p), ("y", C.c_void_p),
                ("alpha", C.c_void_p), ("memkind", C.c_int32), ("reserved", C.c_int32)]


class ials_stats(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("num_users", C.c_int32), ("num_items", C.c_int32),
                ("dim", C.c_int32), ("block", C.c_int32), ("padded_block", C.c_int32),
                ("long_rows_user", C.c_int32), ("long_rows_item", C.c_int32),
                ("segments_user", C.c_int64), ("segments_item", C.c_int64),
                ("fallback_rows", C.c_int64), ("passes", C.c_int64), ("device_bytes", C.c_uint64),
                ("foldin_requests", C.c_int64), ("foldin_float64", C.c_int64),
                ("peak_device_bytes", C.c_uint64), ("solver", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ials_server_config(C.Structure):
    _fields_ = [("num_items", C.c_int32), ("dim", C.c_int32), ("block", C.c_int32), ("alpha0", C.c_float),
                ("lambda_", C.c_float), ("precision", C.c_int32), ("passes", C.c_int32), ("max_slots", C.c_int32),
                ("streams", C.c_int32), ("chol_fallback_ratio", C.c_float), ("hbm_budget", C.c_uint64)]


class ials_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("rejected_busy", C.c_int64), ("completed", C.c_int64),
                ("polled", C.c_int64), ("batches", C.c_int64), ("max_batch", C.c_int64),
                ("float64_requests", C.c_int64), ("not_spd_requests", C.c_int64), ("admitted", C.c_int32),
                ("in_flight", C.c_int32), ("arena_bytes", C.c_uint64), ("bytes_in_use", C.c_uint64),
                ("bytes_peak", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IalsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "ials_create": (C.c_int, [C.POINTER(ials_config), C.POINTER(ials_coo), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(C.c_void_p)]),
    "ials_destroy": (C.c_int, [C.c_void_p]),
    "ials_gramian": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "ials_block_sweep": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "ials_epoch": (C.c_int, [C.c_void_p, C.c_int32]),
    "ials_refresh_predictions": (C.c_int, [C.c_void_p]),
    "ials_loss": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ials_get_csr": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ials_get_predictions": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ials_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ials_stats)]),
    "ials_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ials_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "ials_profile_read": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ials_foldin": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "ials_last_error": (C.c_char_p, [C.c_void_p]),
    "ials_version": (C.c_char_p, []),
    "ials_server_create": (C.c_int, [C.POINTER(ials_server_config), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ials_server_submit": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64]),
    "ials_server_poll": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_int32)]),
    "ials_server_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ials_server_stats)]),
    "ials_server_destroy": (C.c_int, [C.c_void_p]),
    "ials_server_last_error": (C.c_char_p, [C.c_void_p]),
    "ials_rank_topk": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "ials_rank_topk_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                         C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ials_rank_metrics": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ials_rank_last_error": (C.c_char_p, []),
}


def load() -> C.CDLL:
    """Load libials.so (built by paper_2110_14044_amd/build.py).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_14044_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback implementation")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(st: int, ctx=None):
    if st != IALS_OK:
        msg = load().ials_last_error(ctx)
        raise IalsError(st, msg.decode() if msg else "")


def _check_srv(st: int, srv=None):
    if st != IALS_OK:
        msg = load().ials_server_last_error(srv)
        raise IalsError(st, msg.decode() if msg else "")


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a pointer of {type(x)}")


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- one function per C entry point ----

def ials_create(cfg: ials_config, S: ials_coo, W, H, stream=None) -> int:
    out = C.c_void_p()
    st = load().ials_create(C.byref(cfg), C.byref(S), _ptr(W), _ptr(H), _stream(stream), C.byref(out))
    _check(st, None)
    return out.value


def ials_destroy(ctx: int) -> None:
    _check(load().ials_destroy(ctx), None)


def ials_gramian(ctx: int, which: int, block: int, out) -> None:
    _check(load().ials_gramian(ctx, which, block, _ptr(out)), ctx)


def ials_block_sweep(ctx: int, side: int, block: int) -> None:
    _check(load().ials_block_sweep(ctx, side, block), ctx)


def ials_epoch(ctx: int, n_epochs: int) -> None:
    _check(load().ials_epoch(ctx, n_epochs), ctx)


def ials_refresh_predictions(ctx: int) -> None:
    _check(load().ials_refresh_predictions(ctx), ctx)


def ials_loss(ctx: int):
    L = C.c_double()
    parts = (C.c_double * 3)()
    _check(load().ials_loss(ctx, C.byref(L), parts), ctx)
    return L.value, tuple(parts)


def ials_get_csr(ctx: int, side: int, nrows: int, nnz: int):
    ptr = np.zeros(nrows + 1, np.int64)
    col = np.zeros(max(nnz, 1), np.int32)
    perm = np.zeros(max(nnz, 1), np.int32) if side == IALS_SIDE_ITEM else None
    _check(load().ials_get_csr(ctx, side, ptr.ctypes.data, col.ctypes.data,
                               None if perm is None else perm.ctypes.data), ctx)
    return ptr, col[:nnz], (None if perm is None else perm[:nnz])


def ials_get_predictions(ctx: int, nnz: int) -> np.ndarray:
    out = np.zeros(max(nnz, 1), np.float32)
    _check(load().ials_get_predictions(ctx, out.ctypes.data), ctx)
    return out[:nnz]


def ials_get_stats(ctx: int) -> dict:
    s = ials_stats()
    _check(load().ials_get_stats(ctx, C.byref(s)), ctx)
    return s.as_dict()


def ials_set_stream(ctx: int, stream) -> None:
    _check(load().ials_set_stream(ctx, _stream(stream)), ctx)


KERNEL_NAMES = ["predict", "gram_user", "gram_item", "dense_user", "dense_item", "seg_user", "seg_item",
                "rows_user", "rows_item", "fallback_user", "fallback_item", "patch_user", "patch_item", "loss",
                "rows_user_move", "rows_item_move"]


def ials_profile_enable(ctx: int, enable: bool) -> None:
    _check(load().ials_profile_enable(ctx, 1 if enable else 0), ctx)


def ials_profile_read(ctx: int) -> dict:
    ms = np.zeros(16, np.float64)
    cnt = np.zeros(16, np.int64)
    _check(load().ials_profile_read(ctx, ms.ctypes.data, cnt.ctypes.data), ctx)
    return {KERNEL_NAMES[k]: (float(ms[k]), int(cnt[k])) for k in range(16) if cnt[k] > 0}


def ials_foldin(ctx: int, req_ptr: np.ndarray, items, y, passes: int, W_out) -> None:
    """req_ptr: host int64 offsets; items / y / W_out: device tensors (y may be None)."""
    req_ptr = np.ascontiguousarray(req_ptr, np.int64)
    _check(load().ials_foldin(ctx, req_ptr.size - 1, req_ptr.ctypes.data, _ptr(items), _ptr(y), passes,
                              _ptr(W_out)), ctx)


def ials_server_create(cfg: ials_server_config, H) -> int:
    out = C.c_void_p()
    _check_srv(load().ials_server_create(C.byref(cfg), _ptr(H), C.byref(out)), None)
    return out.value


def ials_server_submit(srv: int, items: np.ndarray, y: Optional[np.ndarray], tag: int) -> int:
    """Returns IALS_OK or IALS_E_BUSY; raises on any other status."""
    items = np.ascontiguousarray(items, np.int32)
    yv = None if y is None else np.ascontiguousarray(y, np.float32)
    st = load().ials_server_submit(srv, items.size, items.ctypes.data, None if yv is None else yv.ctypes.data, tag)
    if st not in (IALS_OK, IALS_E_BUSY):
        _check_srv(st, srv)
    return st


def ials_server_poll(srv: int, max_n: int, wait_us: int, d: int):
    """Returns (tags uint64[k], rows float32[k, d], status int32[k])."""
    tags = np.zeros(max(max_n, 1), np.uint64)
    rows = np.zeros((max(max_n, 1), d), np.float32)
    status = np.zeros(max(max_n, 1), np.int32)
    n = C.c_int32()
    _check_srv(load().ials_server_poll(srv, max_n, wait_us, tags.ctypes.data, rows.ctypes.data, status.ctypes.data,
                                       C.byref(n)), srv)
    k = n.value
    return tags[:k], rows[:k], status[:k]


def ials_server_poll_into(srv: int, wait_us: int, tags: np.ndarray, rows: np.ndarray, status: np.ndarray) -> int:
    """Poll into preallocated uint64[m], float32[m, d], int32[m] arrays; returns the count."""
    n = C.c_int32()
    _check_srv(load().ials_server_poll(srv, tags.size, wait_us, tags.ctypes.data, rows.ctypes.data,
                                       status.ctypes.data, C.byref(n)), srv)
    return n.value


def ials_server_stats_get(srv: int) -> dict:
    s = ials_server_stats()
    _check_srv(load().ials_server_stats_get(srv, C.byref(s)), srv)
    return s.as_dict()


def ials_server_destroy(srv: int) -> None:
    _check_srv(load().ials_server_destroy(srv), None)


def ials_server_last_error(srv: Optional[int] = None) -> str:
    m = load().ials_server_last_error(srv)
    return m.decode() if m else ""


def make_server_config(num_items, dim, block, alpha0, lam, passes=3, max_slots=1024, streams=4,
                       hbm_budget=0, chol_fallback_ratio=0.0, precision=IALS_PREC_FP32) -> ials_server_config:
    return ials_server_config(num_items, dim, block, alpha0, lam, precision, passes, max_slots, streams,
                              chol_fallback_ratio, hbm_budget)


def ials_last_error(ctx: Optional[int] = None) -> str:
    m = load().ials_last_error(ctx)
    return m.decode() if m else ""


def ials_version() -> str:
    return load().ials_version().decode()


def make_config(num_users, num_items, dim, block, alpha0, lam, precision=IALS_PREC_FP32,
                chol_fallback_ratio=0.0, hbm_budget=0, flags=0, seg_len=0, gram_split=0) -> ials_config:
    return ials_config(num_users, num_items, dim, block, alpha0, lam, precision, chol_fallback_ratio, flags, seg_len,
                       hbm_budget, gram_split, 0)


def make_coo(user, item, y=None, alpha=None, memkind=IALS_MEM_HOST) -> ials_coo:
    n = int(user.numel() if hasattr(user, "numel") else user.size)
    return ials_coo(n, _ptr(user), _ptr(item), _ptr(y), _ptr(alpha), memkind, 0)


RANK_RECALL = 0
RANK_NDCG = 1


def _check_rank(st: int):
    if st != IALS_OK:
        msg = load().ials_rank_last_error()
        raise IalsError(st, msg.decode() if msg else "")


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    return stream if isinstance(stream, int) else stream.cuda_stream


def ials_rank_topk(W, n_users: int, H, n_items: int, d: int, excl_ptr, excl_idx, k: int, out_ids, out_scores,
                   score_buffer_bytes: int = 0, stream=None) -> None:
    """W, H, excl_ptr, excl_idx, out_ids, out_scores: device tensors (excl_* and out_scores may be None)."""
    _check_rank(load().ials_rank_topk(_ptr(W), n_users, _ptr(H), n_items, d, _ptr(excl_ptr), _ptr(excl_idx), k,
                                      _ptr(out_ids), _ptr(out_scores), score_buffer_bytes, _stream(stream)))


def ials_rank_topk_noalloc(W, n_users: int, H, n_items: int, d: int, excl_ptr, excl_idx, k: int, out_ids,
                           out_scores, stream=None) -> None:
    """ials_rank_topk with the library's fixed score scratch (no device allocation)."""
    _check_rank(load().ials_rank_topk_noalloc(_ptr(W), n_users, _ptr(H), n_items, d, _ptr(excl_ptr),
                                              _ptr(excl_idx), k, _ptr(out_ids), _ptr(out_scores), _stream(stream)))


def ials_rank_metrics(ids, n_users: int, k: int, hold_ptr, hold_idx, kinds, ks, per_user, stream=None):
    """ids, hold_ptr, hold_idx, per_user: device tensors; kinds / ks: sequences of ints.
    Returns (sums float64[m], counts int64[m]) for the m metrics."""
    kinds = np.ascontiguousarray(kinds, np.int32)
    ks = np.ascontiguousarray(ks, np.int32)
    sums = np.zeros(kinds.size, np.float64)
    counts = np.zeros(kinds.size, np.int64)
    _check_rank(load().ials_rank_metrics(_ptr(ids), n_users, k, _ptr(hold_ptr), _ptr(hold_idx), kinds.size,
                                         kinds.ctypes.data, ks.ctypes.data, _ptr(per_user), sums.ctypes.data,
                                         counts.ctypes.data, _stream(stream)))
    return sums, counts
