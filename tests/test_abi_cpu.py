"""C-ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and rejects malformed input before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(cg_\w+)\s*\(", text, re.M))
    return names


@pytest.fixture(scope="module")
def cg():
    from paper_2608_09647_amd import cgmi
    if not os.path.exists(cgmi.LIB_PATH):
        pytest.skip("libcgmi.so not built")
    return cgmi


def test_header_symbols_are_exported(cg):
    declared = _declared_symbols()
    assert {"cg_create", "cg_solve", "cg_spmv", "cg_destroy"} <= declared
    L = cg.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert set(cg.EXPORTED) | set(cg.EXPORTED_FSAI) | set(cg.EXPORTED_BATCH) | set(cg.EXPORTED_IO) == declared


def test_default_opts(cg):
    o = cg.default_opts()
    assert o.precision == cg.PREC_FP64 and o.precond == cg.PC_NONE
    assert o.exchange == cg.EXCHANGE_WHOLE and o.check_every >= 1 and 0 < o.refine_delta < 1
    assert o.vectors == cg.VECTORS_DEVICE


def _create(cg, n, rp, ci, va, rb=0, re=None):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    va = np.ascontiguousarray(va, np.float64)
    code = cg.lib().cg_create(n, int(rp[-1]) if rp.size else 0, rp.ctypes.data, ci.ctypes.data,
                              va.ctypes.data, rb, n if re is None else re, ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("case", ["unsorted", "duplicate", "col_range", "rp_decrease", "rp0",
                                  "range", "neg_n"])
def test_malformed_input_rejected(cg, case):
    rp, ci, va = [0, 2, 3, 5], [0, 1, 1, 0, 2], [4.0, -1.0, 4.0, -1.0, 4.0]
    n, rb, re = 3, 0, 3
    if case == "unsorted":
        ci = [1, 0, 1, 0, 2]
    elif case == "duplicate":
        ci = [0, 0, 1, 0, 2]
    elif case == "col_range":
        ci = [0, 3, 1, 0, 2]
    elif case == "rp_decrease":
        rp = [0, 3, 2, 5]
    elif case == "rp0":
        rp = [1, 2, 3, 5]
    elif case == "range":
        rb, re = 2, 1
    elif case == "neg_n":
        n = -1
    code, h = _create(cg, n, rp, ci, va, rb, re)
    assert code == cg.CG_EINVAL
    assert not h.value
    assert cg.last_error() != ""


def test_destroy_null_is_noop(cg):
    cg.lib().cg_destroy(None)


def test_null_handle_errors(cg):
    r = cg.CgResult()
    assert cg.lib().cg_solve(None, None, None, 1e-10, 10, ctypes.byref(r)) == cg.CG_EINVAL
    assert cg.lib().cg_solve_noalloc(None, None, None, 1e-10, 10, ctypes.byref(r)) == cg.CG_EINVAL
    assert cg.lib().cg_spmv(None, None, None) == cg.CG_EINVAL
    o = cg.default_opts()
    assert cg.lib().cg_set_opts(None, ctypes.byref(o)) == cg.CG_EINVAL


def test_struct_sizes_match_header(cg):
    # cg_opts: 10 x int32 + double + 2 x int32; cg_result: as laid out in include/cgmi.h
    assert ctypes.sizeof(cg.CgOpts) == 56
    assert ctypes.sizeof(cg.CgResult) == 136


def test_product_path_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_2608_09647_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "liboracle" not in text and "cg_oracle" not in text, fn


def test_fsai_entry_points_reject_bad_input(cg):
    L = cg.lib()
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    va = np.array([1.0])
    assert L.cg_set_fsai(None, 1, rp.ctypes.data, ci.ctypes.data, va.ctypes.data) == cg.CG_EINVAL
    assert L.cg_fsai_setup(None, None) == cg.CG_EINVAL
    nnz = ctypes.c_int64()
    assert L.cg_fsai_factor_info(None, ctypes.byref(nnz)) == cg.CG_EINVAL
    t = ctypes.c_void_p()
    theta = np.zeros(cg.FSAI_NPARAMS, np.float32)
    n = np.array([1], np.int32)
    nz = np.array([1], np.int64)
    bad_rp = np.array([1, 1], np.int32)       # row_ptr[0] != 0
    ptr = lambda a: (ctypes.c_void_p * 1)(a.ctypes.data)
    assert L.cg_fsai_trainer_create(1, n.ctypes.data, nz.ctypes.data, ptr(bad_rp), ptr(ci), ptr(va),
                                    theta.ctypes.data, ctypes.byref(t)) == cg.CG_EINVAL
    assert "row_ptr" in cg.last_error()
    assert L.cg_fsai_trainer_create(0, n.ctypes.data, nz.ctypes.data, ptr(rp), ptr(ci), ptr(va),
                                    theta.ctypes.data, ctypes.byref(t)) == cg.CG_EINVAL
    assert L.cg_fsai_train_step(None, 1, None, 1, None, 1e-3, None) == cg.CG_EINVAL
    L.cg_fsai_trainer_destroy(None)


def test_init_params_layout():
    from paper_2608_09647_amd import fsai
    th = fsai.init_params(0)
    assert th.dtype == np.float32 and th.size == 5317
    # biases are zero, weights within the Glorot limits
    assert np.all(th[768:832] == 0) and np.all(th[4928:4992] == 0) and np.all(th[5312:] == 0)
    assert np.abs(th[:768]).max() <= np.sqrt(6 / 76) and np.abs(th[832:4928]).max() <= np.sqrt(6 / 128)
    assert np.array_equal(th, fsai.init_params(0)) and not np.array_equal(th, fsai.init_params(1))


def test_sampling_is_distinct():
    from paper_2608_09647_amd import fsai
    rng = np.random.default_rng(0)
    sys, rows = fsai.sample(rng, [100, 50, 70], 2, 40)
    assert sys.size == 2 and len(set(sys.tolist())) == 2 and rows.shape == (2, 40)
    for s, r in zip(sys, rows):
        assert len(set(r.tolist())) == 40 and r.max() < [100, 50, 70][s]


def test_hbm_copy_rejects_bad_arguments_before_any_device_call(cg):
    L = cg.lib()
    assert L.cg_hbm_copy(None, None, 0, None) == cg.CG_OK
    assert L.cg_hbm_copy(None, None, 5, None) == cg.CG_EINVAL
    assert L.cg_hbm_copy(None, None, -1, None) == cg.CG_EINVAL


def test_host_only_handle_runs_on_host_threads(cg):
    """A host-only handle (rows [0, 0): the paper's CPU-only configuration)
    needs no device: with host vectors its SpMV and CG run on host threads
    alone (also where no GPU is present), the SpMV equal to the oracle's bit
    for bit (rows summed in CSR order), the solve meeting the oracle's bar."""
    import oracle
    from paper_2608_09647_amd import inputs as I
    p = I.poisson3d_problem(16)
    with cg.Solver(p.A, 0, 0) as s:
        s.set_opts(vectors=cg.VECTORS_HOST, host_threads=3)
        x_in = np.random.default_rng(3).uniform(-1, 1, p.A.n)
        y = s.spmv_host(x_in)
        x, res = s.solve_host(p.b, tol=1e-10, maxit=5000)
        rows, nnz = s.slice_info()
    assert rows == 0 and nnz == 0
    assert np.array_equal(y, oracle.spmv(p.A, x_in))
    ref = oracle.cg(p.A, p.b, tol=1e-10, maxit=5000)
    assert res["code"] == cg.CG_OK and res["rows_cpu"] == p.A.n and res["rows_gpu"] == 0
    assert abs(res["iterations"] - ref["iterations"]) <= 2
    true = np.linalg.norm(p.b - oracle.spmv(p.A, x)) / np.linalg.norm(p.b)
    assert true <= 1.01e-10 and abs(res["rel_res_true"] - true) <= 1e-3 * true
    lam = 2 - 2 * np.cos(np.arange(1, 17) * np.pi / 17)
    assert np.linalg.norm(x - ref["x"]) <= 2 * (lam.max() / lam.min()) * 1e-10 * np.linalg.norm(ref["x"])


def test_spmv_kind_range(cg):
    """Tilings 0..7 are accepted (on a host-only handle the choice only takes
    effect once GPU rows exist); anything else is CG_EINVAL."""
    from paper_2608_09647_amd import inputs as I
    A = I.poisson2d(6)
    with cg.Solver(A, 0, 0) as s:
        for k in range(8):
            s.set_opts(spmv_kind=k)
        for bad in (8, -1):
            with pytest.raises(cg.CgError) as e:
                s.set_opts(spmv_kind=bad)
            assert e.value.code == cg.CG_EINVAL and "spmv_kind" in str(e.value)


def test_fuse_dir_values(cg):
    """cg_opts.fuse_dir: automatic by default; CG_FUSE_AUTO, _ON and _OFF are
    accepted, anything else is CG_EINVAL."""
    from paper_2608_09647_amd import inputs as I
    A = I.poisson2d(6)
    with cg.Solver(A, 0, 0) as s:
        assert s.opts.fuse_dir == cg.FUSE_AUTO
        for v in (cg.FUSE_AUTO, cg.FUSE_ON, cg.FUSE_OFF):
            s.set_opts(fuse_dir=v)
        for bad in (3, -1):
            with pytest.raises(cg.CgError) as e:
                s.set_opts(fuse_dir=bad)
            assert e.value.code == cg.CG_EINVAL and "fuse_dir" in str(e.value)
