"""Python binding of libcgmi (C ABI in include/cgmi.h): argument marshalling only.

Every step of the solver runs inside libcgmi.so.  torch provides device
memory and streams; it is imported before the library is loaded so that both
use the same HIP runtime.  Missing library => ImportError-like RuntimeError:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library links against)

# CGMI_LIBRARY: load another build of the library (e.g. a sanitizer build
# from build.py --sanitize) in place of the in-tree libcgmi.so
LIB_PATH = os.environ.get("CGMI_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                           "libcgmi.so")

CG_OK, CG_MAXIT, CG_EINVAL, CG_ENOMEM, CG_EDEVICE, CG_EBREAKDOWN = 0, 1, -1, -2, -3, -4
PREC_FP64, PREC_MIXED = 0, 1
PC_NONE, PC_FSAI = 0, 1
EXCHANGE_WHOLE, EXCHANGE_HALO, EXCHANGE_MAPPED, EXCHANGE_MANAGED = 0, 1, 2, 3
VECTORS_DEVICE, VECTORS_HOST = 0, 1
FUSE_AUTO, FUSE_ON, FUSE_OFF = 0, 1, 2

# Every symbol the public header declares (checked by the tests).
EXPORTED = ["cg_create", "cg_destroy", "cg_set_stream", "cg_default_opts", "cg_set_opts",
            "cg_get_opts", "cg_spmv", "cg_spmv_f32", "cg_solve", "cg_solve_noalloc", "cg_slice_info",
            "cg_read_slice", "cg_hbm_copy", "cg_gather", "cg_last_error"]
NOALLOC_SCRATCH_BYTES = 64 << 20
# include/cgmi_fsai.h
EXPORTED_FSAI = ["cg_fsai_setup", "cg_set_fsai", "cg_fsai_classic", "cg_fsai_factor_info", "cg_fsai_read_factor",
                 "cg_fsai_trainer_create", "cg_fsai_trainer_destroy", "cg_fsai_loss_grad",
                 "cg_fsai_train_step", "cg_fsai_get_params", "cg_fsai_get_state", "cg_fsai_set_state",
                 "cg_fsai_features"]
FSAI_NPARAMS = 5317
# include/cgmi_batch.h
EXPORTED_BATCH = ["cg_batch_create", "cg_batch_destroy", "cg_batch_set_stream", "cg_batch_layout",
                  "cg_batch_default_sched", "cg_batch_set_sched", "cg_batch_get_sched", "cg_batch_solve"]
BATCH_MAX_RHS = 16
BATCH_LAUNCH_COOPERATIVE, BATCH_LAUNCH_ORDINARY = 0, 1
# include/cgmi_io.h
EXPORTED_IO = ["cg_mm_read", "cg_mm_free"]


class MmMatrix(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)), ("col", ctypes.POINTER(ctypes.c_int32)),
                ("val", ctypes.POINTER(ctypes.c_double)), ("symmetric", ctypes.c_int32),
                ("file_entries", ctypes.c_int64)]


class CgOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("exchange", ctypes.c_int32), ("host_threads", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("small_path", ctypes.c_int32), ("spmv_grid", ctypes.c_int32),
                ("spmv_kind", ctypes.c_int32), ("spmv_colblock", ctypes.c_int32),
                ("refine_delta", ctypes.c_double), ("vectors", ctypes.c_int32),
                ("fuse_dir", ctypes.c_int32)]


class CgResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("fp64_residuals", ctypes.c_int32),
                ("rel_res_recur", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("t_solve", ctypes.c_double), ("t_gpu", ctypes.c_double),
                ("t_cpu", ctypes.c_double), ("t_barrier", ctypes.c_double),
                ("t_d2h", ctypes.c_double), ("t_h2d", ctypes.c_double),
                ("t_spmv", ctypes.c_double), ("n_spmv", ctypes.c_int32),
                ("rows_gpu", ctypes.c_int32), ("rows_cpu", ctypes.c_int32),
                ("nnz_gpu", ctypes.c_int64), ("nnz_cpu", ctypes.c_int64),
                ("fell_back", ctypes.c_int32), ("spmv_kind", ctypes.c_int32),
                ("fused_dir", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchSched(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("rows_per_thread", ctypes.c_int32),
                ("team_exponent", ctypes.c_double), ("max_team", ctypes.c_int32),
                ("rhs_per_lane", ctypes.c_int32), ("launch", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("rel_res_recur", ctypes.c_double), ("rel_res_true", ctypes.c_double)]


class BatchStats(ctypes.Structure):
    _fields_ = [("t_kernel", ctypes.c_double), ("grid", ctypes.c_int32),
                ("teams_multi", ctypes.c_int32), ("max_team", ctypes.c_int32),
                ("barriers", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class CgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libcgmi error {code}: {msg}")
        self.code = code


_LIB = None
_vp = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2608_09647_amd.build first")
        L = ctypes.CDLL(LIB_PATH)
        L.cg_create.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_int32,
                                ctypes.c_int32, ctypes.POINTER(_vp)]
        L.cg_create.restype = ctypes.c_int
        L.cg_destroy.argtypes = [_vp]
        L.cg_destroy.restype = None
        L.cg_set_stream.argtypes = [_vp, _vp]
        L.cg_set_stream.restype = ctypes.c_int
        L.cg_default_opts.argtypes = [ctypes.POINTER(CgOpts)]
        L.cg_default_opts.restype = None
        L.cg_set_opts.argtypes = [_vp, ctypes.POINTER(CgOpts)]
        L.cg_set_opts.restype = ctypes.c_int
        L.cg_get_opts.argtypes = [_vp, ctypes.POINTER(CgOpts)]
        L.cg_get_opts.restype = ctypes.c_int
        L.cg_spmv.argtypes = [_vp, _vp, _vp]
        L.cg_spmv.restype = ctypes.c_int
        L.cg_spmv_f32.argtypes = [_vp, _vp, _vp]
        L.cg_spmv_f32.restype = ctypes.c_int
        L.cg_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                               ctypes.POINTER(CgResult)]
        L.cg_solve.restype = ctypes.c_int
        L.cg_solve_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(CgResult)]
        L.cg_solve_noalloc.restype = ctypes.c_int
        L.cg_slice_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
        L.cg_slice_info.restype = ctypes.c_int
        L.cg_read_slice.argtypes = [_vp, _vp, _vp, _vp]
        L.cg_read_slice.restype = ctypes.c_int
        L.cg_last_error.argtypes = []
        L.cg_last_error.restype = ctypes.c_char_p
        L.cg_hbm_copy.argtypes = [_vp, _vp, ctypes.c_int64, _vp]
        L.cg_hbm_copy.restype = ctypes.c_int
        L.cg_gather.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp]
        L.cg_gather.restype = ctypes.c_int
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.cg_fsai_setup.argtypes = [_vp, _vp]
        L.cg_set_fsai.argtypes = [_vp, i64, _vp, _vp, _vp]
        L.cg_fsai_factor_info.argtypes = [_vp, ctypes.POINTER(i64)]
        L.cg_fsai_read_factor.argtypes = [_vp, _vp, _vp, _vp]
        L.cg_fsai_trainer_create.argtypes = [i32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.cg_fsai_trainer_destroy.argtypes = [_vp]
        L.cg_fsai_trainer_destroy.restype = None
        L.cg_fsai_loss_grad.argtypes = [_vp, _vp, i32, _vp, i32, _vp, ctypes.POINTER(dbl), _vp, _vp]
        L.cg_fsai_train_step.argtypes = [_vp, i32, _vp, i32, _vp, dbl, ctypes.POINTER(dbl)]
        L.cg_fsai_get_params.argtypes = [_vp, _vp]
        L.cg_fsai_get_state.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(i32)]
        L.cg_fsai_set_state.argtypes = [_vp, _vp, _vp, _vp, i32]
        L.cg_fsai_features.argtypes = [_vp, i32, _vp]
        L.cg_fsai_classic.argtypes = [_vp]
        for name in EXPORTED_FSAI:
            if name != "cg_fsai_trainer_destroy":
                getattr(L, name).restype = ctypes.c_int
        L.cg_batch_create.argtypes = [i32, _vp, _vp, _vp, _vp, _vp, i32, ctypes.POINTER(_vp)]
        L.cg_batch_destroy.argtypes = [_vp]
        L.cg_batch_destroy.restype = None
        L.cg_batch_set_stream.argtypes = [_vp, _vp]
        L.cg_batch_layout.argtypes = [_vp, _vp]
        L.cg_batch_default_sched.argtypes = [ctypes.POINTER(BatchSched)]
        L.cg_batch_default_sched.restype = None
        L.cg_batch_set_sched.argtypes = [_vp, ctypes.POINTER(BatchSched)]
        L.cg_batch_get_sched.argtypes = [_vp, ctypes.POINTER(BatchSched)]
        L.cg_batch_solve.argtypes = [_vp, _vp, _vp, dbl, i32, _vp, ctypes.POINTER(BatchStats)]
        for name in ("cg_batch_create", "cg_batch_set_stream", "cg_batch_layout", "cg_batch_set_sched",
                     "cg_batch_get_sched", "cg_batch_solve"):
            getattr(L, name).restype = ctypes.c_int
        L.cg_mm_read.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(MmMatrix)]
        L.cg_mm_read.restype = ctypes.c_int
        L.cg_mm_free.argtypes = [ctypes.POINTER(MmMatrix)]
        L.cg_mm_free.restype = None
        _LIB = L
    return _LIB


def last_error() -> str:
    return lib().cg_last_error().decode()


def _check(code: int, allow=(CG_OK,)) -> int:
    if code not in allow:
        raise CgError(code, last_error())
    return code


def default_opts() -> CgOpts:
    o = CgOpts()
    lib().cg_default_opts(ctypes.byref(o))
    return o


def _dev_f32(t, n, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a CUDA float32 tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


def _dev_f64(t, n, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


def _host_f64(a, n, name):
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError(f"{name} must be a C-contiguous float64 numpy array")
    if a.size != n:
        raise ValueError(f"{name} must have {n} elements")
    return ctypes.c_void_p(a.ctypes.data)


class Solver:
    """A cg_handle: the matrix on the GPU row block [row_begin, row_end)."""

    def __init__(self, A, row_begin: int = 0, row_end: int | None = None):
        self.n = int(A.n)
        self._rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        self._ci = np.ascontiguousarray(A.col, dtype=np.int32)
        self._va = np.ascontiguousarray(A.val, dtype=np.float64)
        self.row_begin = int(row_begin)
        self.row_end = self.n if row_end is None else int(row_end)
        h = ctypes.c_void_p()
        _check(lib().cg_create(self.n, int(self._rp[-1]) if self._rp.size else 0,
                               self._rp.ctypes.data, self._ci.ctypes.data, self._va.ctypes.data,
                               self.row_begin, self.row_end, ctypes.byref(h)))
        self._h = h
        del self._rp, self._ci, self._va   # the library holds its own copy
        if self.row_begin < self.row_end or torch.cuda.is_available():
            # the handle's work goes on torch's current stream (a host-only
            # handle without a device has no stream)
            self.set_stream(torch.cuda.current_stream())

    def close(self):
        if getattr(self, "_h", None):
            lib().cg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream):
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        _check(lib().cg_set_stream(self._h, ctypes.c_void_p(ptr)))

    @property
    def opts(self) -> CgOpts:
        o = CgOpts()
        _check(lib().cg_get_opts(self._h, ctypes.byref(o)))
        return o

    def set_opts(self, **kw) -> None:
        o = self.opts
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        _check(lib().cg_set_opts(self._h, ctypes.byref(o)))

    def spmv(self, x, y=None):
        if y is None:
            y = torch.empty_like(x)
        _check(lib().cg_spmv(self._h, _dev_f64(x, self.n, "x"), _dev_f64(y, self.n, "y")))
        return y

    def spmv_f32(self, x, y=None):
        if y is None:
            y = torch.empty_like(x)
        _check(lib().cg_spmv_f32(self._h, _dev_f32(x, self.n, "x"), _dev_f32(y, self.n, "y")))
        return y

    def solve(self, b, x=None, tol: float = 1e-10, maxit: int = 10000, check: bool = True):
        """Solve A x = b in place of x (zeros if None); returns (x, result dict)."""
        if x is None:
            x = torch.zeros_like(b)
        res = CgResult()
        code = lib().cg_solve(self._h, _dev_f64(b, self.n, "b"), _dev_f64(x, self.n, "x"),
                              float(tol), int(maxit), ctypes.byref(res))
        if check:
            _check(code, allow=(CG_OK, CG_MAXIT, CG_EBREAKDOWN))
        out = res.as_dict()
        out["code"] = code
        return x, out

    def solve_noalloc(self, b, x, tol: float = 1e-10, maxit: int = 10000, check: bool = True):
        """cg_solve_noalloc: as solve, with the library's static scratch as the
        only work memory; x (the initial guess, overwritten) must be given."""
        res = CgResult()
        code = lib().cg_solve_noalloc(self._h, _dev_f64(b, self.n, "b"), _dev_f64(x, self.n, "x"),
                                      float(tol), int(maxit), ctypes.byref(res))
        if check:
            _check(code, allow=(CG_OK, CG_MAXIT, CG_EBREAKDOWN))
        out = res.as_dict()
        out["code"] = code
        return x, out

    def spmv_host(self, x, y=None):
        """cg_spmv with host vectors (numpy; needs set_opts(vectors=VECTORS_HOST))."""
        if y is None:
            y = np.empty_like(x)
        _check(lib().cg_spmv(self._h, _host_f64(x, self.n, "x"), _host_f64(y, self.n, "y")))
        return y

    def solve_host(self, b, x=None, tol: float = 1e-10, maxit: int = 10000, check: bool = True):
        """cg_solve with host vectors (numpy; needs set_opts(vectors=VECTORS_HOST)):
        x (zeros if None) is overwritten with the solution."""
        if x is None:
            x = np.zeros_like(b)
        res = CgResult()
        code = lib().cg_solve(self._h, _host_f64(b, self.n, "b"), _host_f64(x, self.n, "x"),
                              float(tol), int(maxit), ctypes.byref(res))
        if check:
            _check(code, allow=(CG_OK, CG_MAXIT, CG_EBREAKDOWN))
        out = res.as_dict()
        out["code"] = code
        return x, out

    def slice_info(self):
        rows = ctypes.c_int32()
        nnz = ctypes.c_int64()
        _check(lib().cg_slice_info(self._h, ctypes.byref(rows), ctypes.byref(nnz)))
        return rows.value, nnz.value

    def read_slice(self):
        rows, nnz = self.slice_info()
        rp = np.empty(rows + 1, np.int32)
        ci = np.empty(max(nnz, 1), np.int32)
        va = np.empty(max(nnz, 1), np.float64)
        _check(lib().cg_read_slice(self._h, rp.ctypes.data, ci.ctypes.data, va.ctypes.data))
        return rp, ci[:nnz], va[:nnz]

    # ---- preconditioner (include/cgmi_fsai.h) --------------------------------
    def set_fsai(self, G) -> None:
        """Install an explicit factor G (CSR with row_ptr/col/val, or scipy CSR):
        M^-1 = G^T G.  Select it with set_opts(precond=PC_FSAI)."""
        rp, ci, va = _csr_arrays(G)
        _check(lib().cg_set_fsai(self._h, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data))

    def fsai_setup(self, theta) -> None:
        """Build the learned factor on the device from the network parameters."""
        th = _params(theta)
        _check(lib().cg_fsai_setup(self._h, th.ctypes.data))

    def fsai_classic(self) -> None:
        """Install the classic (non-learned) FSAI factor on tril(A)."""
        _check(lib().cg_fsai_classic(self._h))

    def read_factor(self):
        nnz = ctypes.c_int64()
        _check(lib().cg_fsai_factor_info(self._h, ctypes.byref(nnz)))
        rp = np.empty(self.n + 1, np.int32)
        ci = np.empty(max(nnz.value, 1), np.int32)
        va = np.empty(max(nnz.value, 1), np.float64)
        _check(lib().cg_fsai_read_factor(self._h, rp.ctypes.data, ci.ctypes.data, va.ctypes.data))
        return rp, ci[:nnz.value], va[:nnz.value]


def _csr_arrays(M):
    if hasattr(M, "indptr"):
        M = M.tocsr()
        M.sort_indices()
        return (np.ascontiguousarray(M.indptr, np.int32), np.ascontiguousarray(M.indices, np.int32),
                np.ascontiguousarray(M.data, np.float64))
    return (np.ascontiguousarray(M.row_ptr, np.int32), np.ascontiguousarray(M.col, np.int32),
            np.ascontiguousarray(M.val, np.float64))


def _params(theta) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float32).reshape(-1)
    if th.size != FSAI_NPARAMS:
        raise ValueError(f"theta must have {FSAI_NPARAMS} entries")
    return th


class FsaiTrainer:
    """Device-resident training set for the learned factor (cg_fsai_trainer)."""

    def __init__(self, systems, theta0):
        self.sizes = [int(A.n) for A in systems]
        arrs = [_csr_arrays(A) for A in systems]
        k = len(arrs)
        n = np.array(self.sizes, np.int32)
        nnz = np.array([int(a[0][-1]) for a in arrs], np.int64)
        ptrs = [(ctypes.c_void_p * k)(*[a[j].ctypes.data for a in arrs]) for j in range(3)]
        th = _params(theta0)
        t = ctypes.c_void_p()
        _check(lib().cg_fsai_trainer_create(k, n.ctypes.data, nnz.ctypes.data, ptrs[0], ptrs[1], ptrs[2],
                                            th.ctypes.data, ctypes.byref(t)))
        self._t = t

    def close(self):
        if getattr(self, "_t", None):
            lib().cg_fsai_trainer_destroy(self._t)
            self._t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _sample(sys, rows):
        sys = np.ascontiguousarray(sys, np.int32).reshape(-1)
        rows = np.ascontiguousarray(rows, np.int32)
        if rows.ndim != 2 or rows.shape[0] != sys.size:
            raise ValueError("rows must have shape (len(sys), rows_per_sys)")
        return sys, rows

    def loss_grad(self, sys, rows, theta=None, outputs: bool = False):
        """(loss, grad[5317]) on the sampled rows (and the network outputs of
        system sys[0], n x 5, if outputs)."""
        sys, rows = self._sample(sys, rows)
        loss = ctypes.c_double()
        grad = np.empty(FSAI_NPARAMS, np.float32)
        out = np.empty((self.sizes[int(sys[0])], 5), np.float32) if outputs else None
        th = None if theta is None else _params(theta)
        _check(lib().cg_fsai_loss_grad(self._t, None if th is None else th.ctypes.data, sys.size,
                                       sys.ctypes.data, rows.shape[1], rows.ctypes.data,
                                       ctypes.byref(loss), grad.ctypes.data,
                                       None if out is None else out.ctypes.data))
        return (loss.value, grad, out) if outputs else (loss.value, grad)

    def step(self, sys, rows, lr: float) -> float:
        sys, rows = self._sample(sys, rows)
        loss = ctypes.c_double()
        _check(lib().cg_fsai_train_step(self._t, sys.size, sys.ctypes.data, rows.shape[1],
                                        rows.ctypes.data, float(lr), ctypes.byref(loss)))
        return loss.value

    def params(self) -> np.ndarray:
        th = np.empty(FSAI_NPARAMS, np.float32)
        _check(lib().cg_fsai_get_params(self._t, th.ctypes.data))
        return th

    def state(self) -> dict:
        """The optimiser state: theta, Adam's m and v (float32) and the step count."""
        th, m, v = (np.empty(FSAI_NPARAMS, np.float32) for _ in range(3))
        step = ctypes.c_int32()
        _check(lib().cg_fsai_get_state(self._t, th.ctypes.data, m.ctypes.data, v.ctypes.data, ctypes.byref(step)))
        return {"theta": th, "m": m, "v": v, "step": int(step.value)}

    def set_state(self, theta, m, v, step: int) -> None:
        arrs = [np.ascontiguousarray(a, np.float32) for a in (theta, m, v)]
        if any(a.size != FSAI_NPARAMS for a in arrs):
            raise ValueError(f"theta, m and v must have {FSAI_NPARAMS} entries")
        _check(lib().cg_fsai_set_state(self._t, *(a.ctypes.data for a in arrs), int(step)))

    def features(self, sys: int) -> np.ndarray:
        f = np.empty((self.sizes[int(sys)], 12), np.float32)
        _check(lib().cg_fsai_features(self._t, int(sys), f.ctypes.data))
        return f


# ---- batched persistent solve (include/cgmi_batch.h) ---------------------------
def default_batch_sched() -> BatchSched:
    s = BatchSched()
    lib().cg_batch_default_sched(ctypes.byref(s))
    return s


class Batch:
    """Many systems x nrhs right-hand sides solved by one persistent launch.
    Vectors are CUDA float64 tensors of shape (n_total, nrhs); system k owns
    rows offsets[k]:offsets[k+1]."""

    def __init__(self, systems, nrhs: int):
        arrs = [_csr_arrays(A) for A in systems]
        k = len(arrs)
        self.nsys, self.nrhs = k, int(nrhs)
        n = np.array([int(A.n) for A in systems], np.int32)
        nnz = np.array([int(a[0][-1]) for a in arrs], np.int64)
        ptrs = [(ctypes.c_void_p * k)(*[a[j].ctypes.data for a in arrs]) for j in range(3)]
        b = ctypes.c_void_p()
        _check(lib().cg_batch_create(k, n.ctypes.data, nnz.ctypes.data, ptrs[0], ptrs[1], ptrs[2],
                                     self.nrhs, ctypes.byref(b)))
        self._b = b
        off = np.empty(k + 1, np.int64)
        _check(lib().cg_batch_layout(self._b, off.ctypes.data))
        self.offsets = off
        self.n_total = int(off[-1])
        self.set_stream(torch.cuda.current_stream())

    def close(self):
        if getattr(self, "_b", None):
            lib().cg_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream):
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        _check(lib().cg_batch_set_stream(self._b, ctypes.c_void_p(ptr)))

    @property
    def sched(self) -> BatchSched:
        s = BatchSched()
        _check(lib().cg_batch_get_sched(self._b, ctypes.byref(s)))
        return s

    def set_sched(self, sched: BatchSched | None = None, **kw) -> None:
        s = self.sched if sched is None else sched
        for key, v in kw.items():
            if not hasattr(s, key):
                raise KeyError(key)
            setattr(s, key, v)
        _check(lib().cg_batch_set_sched(self._b, ctypes.byref(s)))

    def solve(self, B, X=None, tol: float = 1e-10, maxit: int = 10000, check: bool = True):
        """Returns (X, results[nsys, nrhs] as a numpy structured array, stats dict, code)."""
        shape = (self.n_total * self.nrhs,)
        if X is None:
            X = torch.zeros_like(B)
        for t, name in ((B, "B"), (X, "X")):
            if t.dim() != 2 or tuple(t.shape) != (self.n_total, self.nrhs):
                raise ValueError(f"{name} must have shape ({self.n_total}, {self.nrhs})")
        res = (BatchResult * (self.nsys * self.nrhs))()
        st = BatchStats()
        code = lib().cg_batch_solve(self._b, _dev_f64(B.view(-1), shape[0], "B"),
                                    _dev_f64(X.view(-1), shape[0], "X"), float(tol), int(maxit),
                                    res, ctypes.byref(st))
        if check:
            _check(code, allow=(CG_OK, CG_MAXIT, CG_EBREAKDOWN))
        out = np.zeros((self.nsys, self.nrhs), dtype=[("status", np.int32), ("iterations", np.int32),
                                                      ("rel_res_recur", np.float64),
                                                      ("rel_res_true", np.float64)])
        flat = out.reshape(-1)
        for i in range(flat.size):
            flat[i] = (res[i].status, res[i].iterations, res[i].rel_res_recur, res[i].rel_res_true)
        return X, out, st.as_dict(), code


def hbm_copy(src, dst, stream=None) -> None:
    """dst[:] = src[:] with the library's streaming copy kernel (float64
    device tensors of equal length, contiguous); queued on `stream` (a
    torch.cuda.Stream, default: torch's current stream)."""
    n = src.numel()
    if dst.numel() != n:
        raise ValueError("src and dst must have the same length")
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().cg_hbm_copy(_dev_f64(src.view(-1), n, "src"), _dev_f64(dst.view(-1), n, "dst"), n,
                             ctypes.c_void_p(stream.cuda_stream)))


def gather(src, idx, dst, stream=None) -> None:
    """dst[i] = src[idx[i]] with the library's gather kernel (device tensors:
    float64 src and dst, int32 idx; every index must lie inside src)."""
    if not (src.is_cuda and idx.is_cuda and dst.is_cuda) or idx.dtype != torch.int32 \
            or src.dtype != torch.float64 or dst.dtype != torch.float64:
        raise TypeError("src, dst: CUDA float64; idx: CUDA int32")
    if idx.numel() != dst.numel() or not (src.is_contiguous() and idx.is_contiguous() and dst.is_contiguous()):
        raise ValueError("idx and dst must be contiguous with the same length")
    if stream is None:
        stream = torch.cuda.current_stream()
    ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _check(lib().cg_gather(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                           ctypes.c_void_p(dst.data_ptr()), int(idx.numel()), ctypes.c_void_p(ptr)))


def read_matrix_market(path: str, threads: int = 0):
    """Read a Matrix Market coordinate file (real, integer or pattern;
    general or symmetric, symmetric storage expanded) with the library's
    reader; returns (inputs.CSR, info dict)."""
    import numpy as np
    from .inputs import CSR
    m = MmMatrix()
    _check(lib().cg_mm_read(os.fsencode(path), int(threads), ctypes.byref(m)))
    try:
        n, nnz = int(m.n), int(m.nnz)
        rp = np.ctypeslib.as_array(m.row_ptr, shape=(n + 1,)).copy()
        ci = np.ctypeslib.as_array(m.col, shape=(max(nnz, 1),))[:nnz].copy()
        va = np.ctypeslib.as_array(m.val, shape=(max(nnz, 1),))[:nnz].copy()
        info = {"symmetric": bool(m.symmetric), "file_entries": int(m.file_entries)}
    finally:
        lib().cg_mm_free(ctypes.byref(m))
    return CSR(n, rp, ci, va), info
