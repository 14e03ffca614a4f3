"""CPU oracle for the sparse CG hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never links or calls it, and this
package never imports the product package: problems are passed in as plain
arrays (any object with ``n``, ``row_ptr``, ``col``, ``val``).

``cg_oracle.c`` holds the float64 loops (SpMV, CG of Algorithm 1, PCG with
M^{-1} = G^T G, float32-inner CG with float64 reliable updates); this module
loads it with ctypes.  ``fsai.py`` holds the learned-preconditioner oracle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

OK, MAXIT, EINVAL, ENOMEM, EBREAKDOWN = 0, 1, -1, -2, -4

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def lib():
    """Load liboracle.so, building it first only if it is absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_spmv.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_spmv.restype = None
        L.oracle_spmv_f32.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, _f32p, _f32p]
        L.oracle_spmv_f32.restype = None
        L.oracle_dot.argtypes = [ctypes.c_int64, _f64p, _f64p]
        L.oracle_dot.restype = ctypes.c_double
        L.oracle_cg.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p,
                                ctypes.c_double, ctypes.c_int32, _i32p, ctypes.c_void_p, _f64p]
        L.oracle_cg.restype = ctypes.c_int
        L.oracle_pcg.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p,
                                 _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_double,
                                 ctypes.c_int32, _i32p, _f64p]
        L.oracle_pcg.restype = ctypes.c_int
        L.oracle_cg_mixed.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p,
                                      ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                      _i32p, _f64p]
        L.oracle_cg_mixed.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int32]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int32
        _LIB = L
    return _LIB


def _arrs(A):
    return (np.ascontiguousarray(A.row_ptr, dtype=np.int32),
            np.ascontiguousarray(A.col, dtype=np.int32),
            np.ascontiguousarray(A.val, dtype=np.float64))


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def spmv(A, x) -> np.ndarray:
    """y = A x, each row summed left to right in CSR order (Section 3.1)."""
    rp, ci, v = _arrs(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n, dtype=np.float64)
    lib().oracle_spmv(A.n, rp, ci, v, x, y)
    return y


def spmv_f32(A, x32) -> np.ndarray:
    """float32 SpMV on the float32-rounded values of A."""
    rp, ci, v = _arrs(A)
    v32 = v.astype(np.float32)
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    y = np.empty(A.n, dtype=np.float32)
    lib().oracle_spmv_f32(A.n, rp, ci, v32, x32, y)
    return y


def dot(x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(lib().oracle_dot(x.size, x, y))


def cg(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, history: bool = False) -> dict:
    """Unpreconditioned CG of Algorithm 1 with a relative stop test."""
    rp, ci, v = _arrs(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = np.zeros(1, np.int32)
    rr = np.zeros(2)
    hist = np.zeros(maxit + 1) if history else None
    st = lib().oracle_cg(A.n, rp, ci, v, b, x, float(tol), int(maxit), it,
                         hist.ctypes.data if history else None, rr)
    out = {"x": x, "status": int(st), "iterations": int(it[0]),
           "rel_res_recur": float(rr[0]), "rel_res_true": float(rr[1])}
    if history:
        out["rho"] = hist[: int(it[0]) + 1].copy()
    return out


def pcg(A, G, Gt, b, x0=None, tol: float = 1e-10, maxit: int = 10000) -> dict:
    """PCG with z = G^T (G r); G and Gt are explicit CSR matrices."""
    rp, ci, v = _arrs(A)
    grp, gci, gv = _arrs(G)
    trp, tci, tv = _arrs(Gt)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = np.zeros(1, np.int32)
    rr = np.zeros(2)
    st = lib().oracle_pcg(A.n, rp, ci, v, grp, gci, gv, trp, tci, tv, b, x, float(tol),
                          int(maxit), it, rr)
    return {"x": x, "status": int(st), "iterations": int(it[0]),
            "rel_res_recur": float(rr[0]), "rel_res_true": float(rr[1])}


def cg_mixed(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, delta: float = 0.01) -> dict:
    """float32 inner CG with float64 reliable-update refinement."""
    rp, ci, v = _arrs(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    cnt = np.zeros(2, np.int32)
    rr = np.zeros(2)
    st = lib().oracle_cg_mixed(A.n, rp, ci, v, b, x, float(tol), int(maxit), float(delta), cnt, rr)
    return {"x": x, "status": int(st), "iterations": int(cnt[0]), "fp64_residuals": int(cnt[1]),
            "rel_res_recur": float(rr[0]), "rel_res_true": float(rr[1])}


def row_slice(A, row_begin: int, row_end: int):
    """The GPU-owned row block [row_begin, row_end) as (row_ptr rebased, col, val).

    Section 3.2 assigns a contiguous block of rows to the GPU; its CSR is the
    block's rows with row pointers shifted to start at zero.
    """
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    lo, hi = int(rp[row_begin]), int(rp[row_end])
    return ((rp[row_begin:row_end + 1] - lo).astype(np.int32),
            np.asarray(A.col[lo:hi], dtype=np.int32),
            np.asarray(A.val[lo:hi], dtype=np.float64))


def split_rows(n: int, g: float) -> int:
    """n_gpu = round(g * n) (Section 3.2), halves rounded away from zero."""
    x = g * n
    return int(np.floor(x + 0.5)) if x >= 0 else -int(np.floor(-x + 0.5))
