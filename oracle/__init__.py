"""FP64 CPU oracle for iALS++ -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never calls it and shares no code with it; the
two meet only through the seeded inputs of the ``synth`` package.

The arithmetic lives in ``ials_oracle.c`` (plain double-precision C with one
OpenMP loop over independent rows per pass), compiled by ``oracle/build.py``
into ``oracle/libials_oracle.so`` and called here through ctypes.  This module
only marshals numpy arrays.

Functions and the passages they follow:
  build_csr     observation index (the per-user / per-item loops of Alg. 1-3)
  predict       eq. 1, yhat for every observation (Alg. 3, first step of an epoch)
  gramian       eq. 4 (full) and eq. 7 (partial Gramian G^{I,pi}, d x |pi|)
  loss          eq. 2 (all-pairs term through <W^T W, H^T H>_F)
  block_pass    one (block, side) pass of Alg. 3 given G (eq. 8-9 and the update)
  epochs        Alg. 3, T epochs, users then items inside each block
  foldin        the user-side block step of Alg. 3 for one new row with H fixed,
                repeated for a number of sweeps (eq. 3 is its b = d, one-sweep limit)

Pins (tests/test_oracle_pins.py): CSR vs numpy lexsort; loss vs the all-pairs
sum; block step vs scipy minimisation and a zero block gradient by finite
differences; b = d vs eq. 3 solved with numpy.linalg.solve (Alg. 1); b = 1 vs an
independently written Alg. 2 (iCD); monotone loss; fold-in vs eq. 3.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# IALS_ORACLE_LIB selects another build of the same source (the sanitizer tests use it)
LIB_PATH = os.environ.get("IALS_ORACLE_LIB") or os.path.join(_HERE, "libials_oracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class _Nullable:
    """ctypes argtype accepting a float64 array or None."""

    @classmethod
    def from_param(cls, obj):
        if obj is None:
            return None
        if not (isinstance(obj, np.ndarray) and obj.dtype == np.float64 and obj.flags.c_contiguous):
            raise TypeError("expected C-contiguous float64 array or None")
        return obj.ctypes.data_as(C.c_void_p)


class _NullableI32:
    @classmethod
    def from_param(cls, obj):
        if obj is None:
            return None
        if not (isinstance(obj, np.ndarray) and obj.dtype == np.int32 and obj.flags.c_contiguous):
            raise TypeError("expected C-contiguous int32 array or None")
        return obj.ctypes.data_as(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.ora_build_csr.argtypes = [C.c_int64, C.c_int32, C.c_int32, _i32p, _i32p, _i64p, _i32p, _i64p]
        L.ora_build_csr.restype = C.c_int
        L.ora_predict.argtypes = [C.c_int32, C.c_int32, _i64p, _i32p, _f64p, _f64p, _f64p]
        L.ora_predict.restype = None
        L.ora_gramian.argtypes = [C.c_int32, C.c_int32, _f64p, C.c_int32, C.c_int32, _f64p]
        L.ora_gramian.restype = None
        L.ora_loss.argtypes = [C.c_int32, C.c_int32, C.c_int32, _i64p, _i32p, _Nullable, _Nullable,
                               _f64p, _f64p, C.c_double, C.c_double, _Nullable]
        L.ora_loss.restype = C.c_double
        L.ora_pass.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                               _i64p, _i32p, _NullableI32, _Nullable, _Nullable, _f64p, _f64p, _f64p,
                               _f64p]
        L.ora_pass.restype = C.c_int64
        L.ora_pass_rows.argtypes = [C.c_int32, _i32p, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                               _i64p, _i32p, _NullableI32, _Nullable, _Nullable, _f64p, _f64p, _f64p,
                               _f64p]
        L.ora_pass_rows.restype = C.c_int64
        L.ora_epochs.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                 _i64p, _i32p, _i64p, _i32p, _i32p, _Nullable, _Nullable, _f64p,
                                 _f64p, _f64p, C.c_int32, _Nullable]
        L.ora_epochs.restype = C.c_int
        L.ora_foldin.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, _f64p,
                                 _f64p, C.c_int32, _i64p, _i32p, _Nullable, C.c_int32, _f64p]
        L.ora_foldin.restype = C.c_int
        _lib = L
    return _lib


def _f64(x):
    return None if x is None else np.ascontiguousarray(x, dtype=np.float64)


class CSR:
    """user-CSR (yhat order) and item-CSR with perm[item slot] = user slot."""

    def __init__(self, num_users, num_items, uptr, ucol, usrc, iptr, icol, perm):
        self.num_users, self.num_items = num_users, num_items
        self.uptr, self.ucol, self.usrc = uptr, ucol, usrc
        self.iptr, self.icol, self.perm = iptr, icol, perm


def build_csr_side(nrows: int, ncols: int, row: np.ndarray, col: np.ndarray):
    row = np.ascontiguousarray(row, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    nnz = row.size
    ptr = np.zeros(nrows + 1, np.int64)
    col_out = np.zeros(max(nnz, 1), np.int32)
    src = np.zeros(max(nnz, 1), np.int64)
    st = lib().ora_build_csr(nnz, nrows, ncols, row, col, ptr, col_out, src)
    if st != 0:
        raise ValueError(f"invalid observations (status {st})")
    return ptr, col_out[:nnz], src[:nnz]


def build_csr(num_users: int, num_items: int, user: np.ndarray, item: np.ndarray) -> CSR:
    uptr, ucol, usrc = build_csr_side(num_users, num_items, user, item)
    iptr, icol, isrc = build_csr_side(num_items, num_users, item, user)
    pos = np.empty(usrc.size, np.int64)
    pos[usrc] = np.arange(usrc.size, dtype=np.int64)
    perm = pos[isrc].astype(np.int32)
    return CSR(num_users, num_items, uptr, ucol, usrc, iptr, icol, perm)


def predict(csr: CSR, W: np.ndarray, H: np.ndarray) -> np.ndarray:
    W, H = _f64(W), _f64(H)
    out = np.zeros(csr.ucol.size, np.float64)
    lib().ora_predict(csr.num_users, W.shape[1], csr.uptr, csr.ucol, W, H, out)
    return out


def gramian(X: np.ndarray, p0: int = 0, bw: Optional[int] = None) -> np.ndarray:
    X = _f64(X)
    n, d = X.shape
    bw = d - p0 if bw is None else bw
    G = np.zeros((d, bw), np.float64)
    lib().ora_gramian(n, d, X, p0, bw, G)
    return G


def loss(csr: CSR, W, H, alpha0: float, lam: float, y=None, a=None, parts: bool = False):
    W, H = _f64(W), _f64(H)
    p = np.zeros(3, np.float64)
    L = lib().ora_loss(csr.num_users, csr.num_items, W.shape[1], csr.uptr, csr.ucol, _f64(y), _f64(a),
                       W, H, alpha0, lam, p)
    return (L, p) if parts else L


def to_slot_order(csr: CSR, v: Optional[np.ndarray]) -> Optional[np.ndarray]:
    """Reorder a per-observation array from input (COO) order to user-CSR slot order."""
    return None if v is None else np.ascontiguousarray(np.asarray(v, np.float64)[csr.usrc])


def block_pass(csr: CSR, side: str, p0: int, bw: int, alpha0: float, lam: float, W: np.ndarray,
               H: np.ndarray, yhat: np.ndarray, G: np.ndarray, y=None, a=None) -> int:
    """In place: one pass over 'user' or 'item' rows for block [p0, p0+bw) given G (d x bw)."""
    d = W.shape[1]
    G = _f64(G)
    if side == "user":
        return lib().ora_pass(csr.num_users, d, p0, bw, alpha0, lam, csr.uptr, csr.ucol, None, y, a,
                              W, H, G, yhat)
    return lib().ora_pass(csr.num_items, d, p0, bw, alpha0, lam, csr.iptr, csr.icol, csr.perm, y, a,
                          H, W, G, yhat)


def pass_rows(csr: CSR, side: str, rows, p0: int, bw: int, alpha0: float, lam: float, W: np.ndarray,
              H: np.ndarray, yhat: np.ndarray, G: np.ndarray, y=None, a=None) -> int:
    """In place: the block step of the listed rows only (each exactly as in block_pass)."""
    d = W.shape[1]
    G = _f64(G)
    rows = np.ascontiguousarray(rows, np.int32)
    if side == "user":
        return lib().ora_pass_rows(rows.size, rows, d, p0, bw, alpha0, lam, csr.uptr, csr.ucol,
                                   None, y, a, W, H, G, yhat)
    return lib().ora_pass_rows(rows.size, rows, d, p0, bw, alpha0, lam, csr.iptr, csr.icol, csr.perm, y, a,
                               H, W, G, yhat)


def epochs(csr: CSR, W0, H0, b: int, alpha0: float, lam: float, n_epochs: int, y=None, a=None):
    """Run n_epochs of Alg. 3 from (W0, H0).  y, a are in user-CSR slot order.
    Returns (W, H, yhat, loss per epoch)."""
    W = np.array(W0, dtype=np.float64, order="C", copy=True)
    H = np.array(H0, dtype=np.float64, order="C", copy=True)
    d = W.shape[1]
    yhat = np.zeros(csr.ucol.size, np.float64)
    losses = np.zeros(max(n_epochs, 1), np.float64)
    st = lib().ora_epochs(csr.num_users, csr.num_items, d, b, alpha0, lam, csr.uptr, csr.ucol, csr.iptr,
                          csr.icol, csr.perm, _f64(y), _f64(a), W, H, yhat, n_epochs, losses)
    if st != 0:
        raise RuntimeError(f"oracle epochs failed with status {st}")
    return W, H, yhat, losses[:n_epochs]


def foldin(H, b: int, alpha0: float, lam: float, req_ptr, items, passes: int, y=None, GH=None):
    H = _f64(H)
    I, d = H.shape
    GH = gramian(H) if GH is None else _f64(GH)
    req_ptr = np.ascontiguousarray(req_ptr, np.int64)
    items = np.ascontiguousarray(items, np.int32)
    n = req_ptr.size - 1
    out = np.zeros((n, d), np.float64)
    st = lib().ora_foldin(I, d, b, alpha0, lam, H, GH, n, req_ptr, items, _f64(y), passes, out)
    if st != 0:
        raise RuntimeError(f"oracle fold-in failed with status {st}")
    return out
