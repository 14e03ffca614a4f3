"""GPU parity: libcgmi (C ABI, HIP kernels) against the CPU oracle.

Bars (derived from the arithmetic):
* SpMV: max_i |y_i - yhat_i| / sum_k |a_ik x_k| <= 1e-12 (sum-order bound for
  rows of up to ~2000 nonzeros is ~2.3e-13); bit-exact on integer inputs.
* Row split / device slice: bit-exact.
* CG: both sides converge, true relative residual <= tol (checked with the
  oracle's own SpMV on the GPU's x), iteration counts within max(2, 2%),
  ||x_gpu - x_oracle|| / ||x_oracle|| <= 2 kappa tol.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2608_09647_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cg(require_gpu):
    from paper_2608_09647_amd import cgmi
    cgmi.lib()
    return cgmi


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def managed_supported(cg) -> bool:
    """Managed memory for p needs the device to report managed-memory
    support (XNACK-off MI355X systems report none: the library then returns
    CG_EINVAL for CG_EXCHANGE_MANAGED)."""
    with cg.Solver(I.poisson2d(4)) as s:
        try:
            s.set_opts(exchange=cg.EXCHANGE_MANAGED)
            return True
        except cg.CgError as e:
            assert "managed-memory support" in str(e)
            return False


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def arrowhead(n, seed=0):
    """SPD arrowhead: row/column 0 dense (exercises the workgroup-per-row bin)."""
    rng = np.random.default_rng(seed)
    M = sp.lil_matrix((n, n))
    v = -rng.random(n - 1) / n
    M[0, 1:] = v
    M[1:, 0] = v[:, None]
    M.setdiag(np.concatenate([[2.0], 1.0 + rng.random(n - 1)]))
    S = M.tocsr()
    S.sort_indices()
    return I.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


def spmv_err(A, x, y, ref):
    absA = sp.csr_matrix((np.abs(A.val), A.col, A.row_ptr), shape=(A.n, A.n))
    scale = absA @ np.abs(x)
    scale[scale == 0] = 1e-300
    return float(np.max(np.abs(y - ref) / scale))


SPMV_CASES = {
    "poisson2d_64": lambda: I.poisson2d(64),
    "poisson3d_24": lambda: I.poisson3d(24),
    "poisson3d_ragged": lambda: I.poisson3d(13, 11, 7),
    "poisson3d_planes_256": lambda: I.poisson3d(256, 256, 3),   # column gaps up to 65,536
    "random_spd_30k": lambda: I.random_spd_lognormal(30000, seed=3),
    "diffusion_100": lambda: I.diffusion2d(I.log_normal_field(100, 100, [1, 0])),
    "arrowhead_3000": lambda: arrowhead(3000),
    "tiny_1": lambda: I.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5])),
    "tiny_7": lambda: I.poisson2d(7, 1),
}


@pytest.mark.parametrize("name", list(SPMV_CASES))
def test_spmv_matches_oracle(cg, name):
    A = SPMV_CASES[name]()
    print(f"[spmv] {name} n={A.n} nnz={A.nnz}", flush=True)
    x = np.random.default_rng(7).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    with cg.Solver(A) as s:
        y = host(s.spmv(dev(x)))
    assert spmv_err(A, x, y, ref) <= 1e-12
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12 * (np.abs(ref).max() + 1))


def used_kind(s, n):
    """The tiling the solver runs (reported by a solve that stops at once)."""
    _, res = s.solve(dev(np.ones(n)), tol=0.0, maxit=0, check=False)
    return res["spmv_kind"]


def stencil_applies(A):
    """Whether every 64-row slice has at most 8 distinct column offsets
    (column - row), so stencil slices (kind 6) apply."""
    lens = np.diff(A.row_ptr)
    if lens.max() > 8:
        return False
    rows = np.repeat(np.arange(A.n), lens)
    off = A.col.astype(np.int64) - rows
    for t in range(0, A.n, 64):
        o = off[A.row_ptr[t]:A.row_ptr[min(A.n, t + 64)]]
        if np.unique(o).size > 8:
            return False
    return True


def gaps_apply(A):
    """Whether gap-coded slices (kind 7) apply: rows of at most 8 entries,
    consecutive columns at most 2^16 apart, and every row's first column
    within 2^19 of its own index (20-bit two's complement offsets)."""
    lens = np.diff(A.row_ptr)
    if lens.max() > 8:
        return False
    d = np.diff(A.col.astype(np.int64))
    inner = np.ones(A.nnz, bool)
    inner[A.row_ptr[:-1][lens > 0]] = False   # each row's first entry has no gap
    d = d[inner[1:]]
    if not np.all((d >= 1) & (d <= 65536)):
        return False
    rows = np.flatnonzero(lens > 0)
    off = A.col[A.row_ptr[rows]].astype(np.int64) - rows
    return bool(np.all((off >= -(1 << 19)) & (off < (1 << 19))))


@pytest.mark.parametrize("kind", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("name", ["poisson2d_64", "poisson3d_ragged", "diffusion_100", "tiny_7",
                                  "random_spd_30k", "tiny_1"])
def test_spmv_tilings_match_oracle(cg, name, kind):
    A = SPMV_CASES[name]()
    x = np.random.default_rng(11).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    with cg.Solver(A) as s:
        s.set_opts(spmv_kind=kind)
        y = host(s.spmv(dev(x)))
        used = used_kind(s, A.n)
    assert spmv_err(A, x, y, ref) <= 1e-12
    if kind in (2, 3) and s_kind_used(A, kind):
        assert used == kind
    if kind == 4:
        assert used == (4 if np.diff(A.row_ptr).max() <= 8 else 3 if np.diff(A.row_ptr).max() <= 64 else 1)
    if kind == 5:
        assert used == 5
    if kind == 6 and stencil_applies(A):
        assert used == 6
    if kind == 7:
        assert used == (7 if gaps_apply(A) else 3 if np.diff(A.row_ptr).max() <= 64 else 1)
    if used in (2, 3, 4, 6, 7):
        # stream, sliced (plain or gap-coded columns), dictionary-sliced and
        # stencil tiles sum each row left to right with rounded products: the
        # oracle's own order, so the bits agree
        assert np.array_equal(y, ref)


@pytest.mark.parametrize("cols", [97, 1000, 4096])
@pytest.mark.parametrize("name", ["random_spd_30k", "arrowhead_3000", "poisson3d_ragged"])
def test_column_blocks_match_oracle(cg, name, cols):
    """Column blocks of `cols` columns (many blocks on small matrices), each
    walked in natural row order with lanes for half its mean row length; the
    arrowhead's dense row loops in its lane group."""
    A = SPMV_CASES[name]()
    x = np.random.default_rng(5).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    if (A.n + cols - 1) // cols > 64:
        cols = (A.n + 63) // 64
    with cg.Solver(A) as s:
        s.set_opts(spmv_kind=5, spmv_colblock=cols)
        y = host(s.spmv(dev(x)))
        assert used_kind(s, A.n) == 5
    assert spmv_err(A, x, y, ref) <= 1e-12


@pytest.mark.parametrize("cols", [5000, 8192])
def test_column_blocks_with_a_huge_row_keep_length_bins(cg, cols):
    """A block holding a row longer than 4096 entries keeps the length bins,
    where that row is reduced by a whole workgroup."""
    A = arrowhead(6000, seed=3)
    x = np.random.default_rng(6).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    with cg.Solver(A) as s:
        s.set_opts(spmv_kind=5, spmv_colblock=cols)
        y = host(s.spmv(dev(x)))
        assert used_kind(s, A.n) == 5
    assert spmv_err(A, x, y, ref) <= 1e-12


def test_column_blocks_cg_mixed_and_split(cg):
    p = I.random_spd_problem(20000, seed=3)
    ref = oracle.cg(p.A, p.b, tol=1e-10, maxit=20000)
    refm = oracle.cg_mixed(p.A, p.b, tol=1e-10, maxit=20000)
    for opts in ({}, {"precision": cg.PREC_MIXED}):
        with cg.Solver(p.A) as s:
            s.set_opts(spmv_kind=5, spmv_colblock=3000, **opts)
            x, res = s.solve(dev(p.b), tol=1e-10, maxit=20000)
        r = refm if opts else ref
        print(f"[colblock] {opts} it={res['iterations']} oracle={r['iterations']}", flush=True)
        assert res["code"] == cg.CG_OK and res["spmv_kind"] == 5
        assert abs(res["iterations"] - r["iterations"]) <= max(2, 0.05 * r["iterations"])
        true = np.linalg.norm(p.b - oracle.spmv(p.A, host(x))) / np.linalg.norm(p.b)
        assert true <= 1.01e-10
    # split rows: the GPU block [rb, re) with global columns split into blocks
    n = p.A.n
    with cg.Solver(p.A, 5000, 15000) as s:
        s.set_opts(spmv_kind=5, spmv_colblock=4000)
        x, res = s.solve(dev(p.b), tol=1e-10, maxit=20000)
    assert res["code"] == cg.CG_OK
    assert abs(res["iterations"] - ref["iterations"]) <= max(2, 0.05 * ref["iterations"])
    assert np.linalg.norm(p.b - oracle.spmv(p.A, host(x))) / np.linalg.norm(p.b) <= 1.01e-10


def test_dictionary_slices_fall_back_on_many_offsets(cg):
    """Rows of <= 8 entries whose 64-row slices use more than 15 distinct
    column offsets take plain slices."""
    n = 4096
    rng = np.random.default_rng(2)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for _ in range(2):          # two random perfect matchings: rows of <= 3 entries
        perm = rng.permutation(n)
        a, b = perm[0::2], perm[1::2]
        rows += [a, b]
        cols += [b, a]
    r, cidx = np.concatenate(rows), np.concatenate(cols)
    v = np.where(r == cidx, 8.0, -0.5)
    S = sp.csr_matrix((v, (r, cidx)), shape=(n, n))
    S.sum_duplicates()
    S.sort_indices()
    assert np.diff(S.indptr).max() <= 8
    A = I.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    x = rng.uniform(-1, 1, n)
    with cg.Solver(A) as s:
        s.set_opts(spmv_kind=4)
        assert used_kind(s, n) == 3
        assert np.array_equal(host(s.spmv(dev(x))), oracle.spmv(A, x))


def s_kind_used(A, kind):
    """Whether the requested tiling applies (otherwise vector bins are used)."""
    lens = np.diff(A.row_ptr)
    if kind == 3:
        return lens.max() <= 64
    # stream tiles: every row's entries fit one tile (512 slots from the
    # row's first entry rounded down to a multiple of 4)
    rp = A.row_ptr.astype(np.int64)
    return bool(np.all((rp[:-1] & 3) + np.diff(rp) <= 512))


@pytest.mark.parametrize("name", ["poisson3d_ragged", "random_spd_30k", "arrowhead_3000"])
def test_spmv_integer_inputs_bitwise(cg, name):
    A = SPMV_CASES[name]()
    A.val = np.rint(A.val * 16.0)            # small integers: every partial sum is exact
    x = np.random.default_rng(3).integers(-1000, 1001, A.n).astype(np.float64)
    ref = oracle.spmv(A, x)
    with cg.Solver(A) as s:
        y = host(s.spmv(dev(x)))
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("rb,re", [(0, None), (100, 900), (0, 1), (1, 1000), (999, 1000), (500, 500)])
def test_device_slice_bit_exact(cg, rb, re):
    A = I.random_spd_lognormal(1000, seed=9)
    re = A.n if re is None else re
    with cg.Solver(A, rb, re) as s:
        rows, nnz = s.slice_info()
        assert rows == re - rb and nnz == A.row_ptr[re] - A.row_ptr[rb]
        rp, ci, va = s.read_slice()
    orp, oci, ova = oracle.row_slice(A, rb, re)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci) and np.array_equal(va, ova)


def kappa_of(name, A):
    """Condition number: closed forms for the Laplacians, Gershgorin over the
    exact smallest eigenvalue 0.01 for the random diagonally dominant family,
    Lanczos for the diffusion operator."""
    if name.startswith("poisson"):
        N = round(A.n ** (1 / (3 if "3d" in name else 2)))
        lam = 2 - 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
        return lam.max() / lam.min()
    if name.startswith("random_spd"):
        return np.max(np.add.reduceat(np.abs(A.val), A.row_ptr[:-1])) / 0.01
    S = A.scipy()
    lmax = spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    lmin = spla.eigsh(S, k=1, sigma=0, which="LM", return_eigenvectors=False, tol=1e-6)[0]
    return lmax / lmin


CG_CASES = {
    "poisson2d_64": lambda: I.poisson2d_problem(64),
    "poisson3d_32": lambda: I.poisson3d_problem(32),
    "diffusion_64": lambda: I.diffusion_problem(64, seed=10_000),
    "random_spd_20k": lambda: I.random_spd_problem(20000, seed=3),
}


def check_cg(A, b, x_gpu, res, ref, tol, kappa):
    assert res["status"] == oracle.OK and ref["status"] == oracle.OK
    true = np.linalg.norm(b - oracle.spmv(A, x_gpu)) / np.linalg.norm(b)
    assert true <= tol * 1.01, true
    assert abs(res["rel_res_true"] - true) <= 1e-3 * true + 1e-16
    # finite-precision CG: the step at which tol is crossed moves with the
    # summation order; a few percent at kappa ~ 1e5..1e6
    assert abs(res["iterations"] - ref["iterations"]) <= max(2, 0.05 * ref["iterations"])
    err = np.linalg.norm(x_gpu - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 2 * kappa * tol, (err, kappa)


@pytest.mark.parametrize("small_path", [1, 0])
@pytest.mark.parametrize("name", list(CG_CASES))
def test_cg_matches_oracle(cg, name, small_path):
    p = CG_CASES[name]()
    print(f"[cg] {name} n={p.A.n} small_path={small_path}", flush=True)
    ref = oracle.cg(p.A, p.b, tol=1e-10, maxit=20000)
    with cg.Solver(p.A) as s:
        s.set_opts(small_path=small_path)
        x, res = s.solve(dev(p.b), tol=1e-10, maxit=20000)
    check_cg(p.A, p.b, host(x), res, ref, 1e-10, kappa_of(name, p.A))



# One case per single-workgroup variant: rows per thread (n up to 1024, 2048,
# 4096) x longest row (register-resident rows up to 8 / 20, 8 / 12, 5 entries,
# else the CSR variant that reads the rows from memory at every product).
# The random matrices take diagonal shift 1 (condition numbers of a few
# hundred).  Fixed-work iterates are compared against the oracle's with a bar
# of 4x the distance between two other correct float64 CGs (the oracle's and
# one with scipy products and BLAS dots): rows of hundreds of entries whose
# diagonal cancels their off-diagonal sum move the iterates by ~1e-9 under a
# mere change of summation order.
SMALL_CASES = {
    "rpt1_len5": (1, 5, 5, "poisson2d", lambda: I.poisson2d(30)),
    "rpt1_len9_20": (1, 9, 20, "random", lambda: I.random_spd_lognormal(1000, 1, mean_degree=5, sigma=0.3,
                                                                      max_degree=6, shift=1.0)),
    "rpt1_csr": (1, 21, 10**9, "random", lambda: I.random_spd_lognormal(1000, 0, shift=1.0)),
    "rpt2_len7": (2, 1, 8, "poisson3d", lambda: I.poisson3d(12)),
    "rpt2_len9_12": (2, 9, 12, "random", lambda: I.random_spd_lognormal(2000, 1, mean_degree=2, sigma=0.2,
                                                                      max_degree=3, shift=1.0)),
    "rpt2_csr": (2, 13, 10**9, "random", lambda: I.random_spd_lognormal(2000, 0, shift=1.0)),
    "rpt4_len5": (4, 1, 5, "poisson2d", lambda: I.poisson2d(60)),
    "rpt4_csr": (4, 6, 10**9, "poisson3d", lambda: I.poisson3d(15)),
}


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_small_path_variants_match_oracle(cg, name):
    rpt, lo, hi, family, make = SMALL_CASES[name]
    A = make()
    L = int(np.diff(A.row_ptr).max())
    assert -(-A.n // 1024) == rpt and lo <= L <= hi, (A.n, L)   # the case reaches the intended variant
    xs = I.uniform_vector(A.n, [17, 1])
    b = I.rhs_of(A, xs)
    print(f"[small] {name} n={A.n} longest row {L}", flush=True)
    if family == "random":   # diagonal shift 1: smallest eigenvalue 1, Gershgorin above
        kappa = np.max(np.add.reduceat(np.abs(A.val), A.row_ptr[:-1]))
    else:
        kappa = kappa_of(family, A)
    ref = oracle.cg(A, b, tol=1e-10, maxit=20000)
    fixed = oracle.cg(A, b, tol=0.0, maxit=30)
    S = A.scipy()
    xa, r, rho = np.zeros(A.n), b.copy(), b @ b
    pa = r.copy()
    for _ in range(30):
        q = S @ pa
        alpha = rho / (pa @ q)
        xa += alpha * pa
        r -= alpha * q
        rho, rho_old = r @ r, rho
        pa = r + (rho / rho_old) * pa
    spread = np.linalg.norm(xa - fixed["x"]) / np.linalg.norm(fixed["x"])
    spread_res = abs(np.sqrt(rho) / np.linalg.norm(b) - fixed["rel_res_recur"]) / fixed["rel_res_recur"]
    with cg.Solver(A) as s:
        s.set_opts(small_path=1)
        x, res = s.solve(dev(b), tol=1e-10, maxit=20000)
        check_cg(A, b, host(x), res, ref, 1e-10, kappa)
        x, res = s.solve(dev(b), tol=0.0, maxit=30)
        assert res["iterations"] == 30 and res["status"] == oracle.MAXIT
        x = host(x)
        assert np.linalg.norm(x - fixed["x"]) / np.linalg.norm(fixed["x"]) <= max(1e-11, 4 * spread), spread
        assert (abs(res["rel_res_recur"] - fixed["rel_res_recur"])
                <= max(1e-8, 4 * spread_res) * fixed["rel_res_recur"]), spread_res


def test_cg_fixed_work_tracks_oracle(cg):
    p = I.poisson3d_problem(32)
    ref = oracle.cg(p.A, p.b, tol=0.0, maxit=60)
    with cg.Solver(p.A) as s:
        x, res = s.solve(dev(p.b), tol=0.0, maxit=60)
    assert res["iterations"] == 60 and res["status"] == oracle.MAXIT
    x = host(x)
    assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-11
    assert abs(res["rel_res_recur"] - ref["rel_res_recur"]) <= 1e-6 * ref["rel_res_recur"]


@pytest.mark.parametrize("exchange", [0, 1, 2, 3])
@pytest.mark.parametrize("frac", [0.0, 0.5, 1.0, "mid"])
def test_split_modes_match_oracle(cg, frac, exchange):
    if exchange == 3 and not managed_supported(cg):
        pytest.skip("the device reports no managed-memory support")
    p = I.poisson3d_problem(20)
    n = p.A.n
    if frac == "mid":
        rb, re = n // 4, (3 * n) // 4
    else:
        rb, re = 0, oracle.split_rows(n, frac)
    print(f"[split] rows [{rb},{re}) of {n}, exchange={exchange}", flush=True)
    ref = oracle.cg(p.A, p.b, tol=1e-10, maxit=5000)
    with cg.Solver(p.A, rb, re) as s:
        s.set_opts(exchange=exchange, host_threads=4)
        x, res = s.solve(dev(p.b), tol=1e-10, maxit=5000)
    assert res["rows_gpu"] == re - rb and res["rows_cpu"] == n - (re - rb)
    assert res["nnz_gpu"] + res["nnz_cpu"] == p.A.nnz
    if 0 < re - rb < n:   # GPU phases timed by events on the stream: within the solve's wall time
        assert 0.0 < res["t_gpu"] < res["t_solve"]
    lam = 2 - 2 * np.cos(np.arange(1, 21) * np.pi / 21)
    check_cg(p.A, p.b, host(x), res, ref, 1e-10, lam.max() / lam.min())


def test_split_memory_modes_agree_bitwise(cg):
    """Explicit copies (whole, halo), mapped host memory and managed memory
    only change where p lives: the same kernels and host loops see the same
    values, so the iterates agree bit for bit."""
    p = I.random_spd_problem(8000, seed=4)
    xs = []
    for exchange in (0, 1, 2, 3) if managed_supported(cg) else (0, 1, 2):
        with cg.Solver(p.A, 0, 5000) as s:
            s.set_opts(exchange=exchange, host_threads=3)
            x, res = s.solve(dev(p.b), tol=1e-10, maxit=3000)
            xs.append((host(x), res["iterations"]))
            if exchange >= 2:
                assert res["t_d2h"] < 0.5 and res["t_h2d"] < 0.5   # only the initial/final transfers
    for xk, it in xs[1:]:
        assert it == xs[0][1] and np.array_equal(xk, xs[0][0])


@pytest.mark.parametrize("n_side", [24, 40])   # 576 rows (small-path size), 64,000 rows
def test_gpu_only_shared_p_modes_bitwise(cg, n_side):
    """GPU-only handles with p in mapped or managed memory run the
    multi-kernel iteration on that memory: bitwise equal to the device-memory
    solve with the single-workgroup path off."""
    p = I.poisson2d_problem(n_side) if n_side == 24 else I.poisson3d_problem(n_side)
    out = {}
    modes = (0, 2, 3, 0) if managed_supported(cg) else (0, 2, 0)
    with cg.Solver(p.A) as s:
        for exchange in modes:
            s.set_opts(exchange=exchange, small_path=0)
            x, res = s.solve(dev(p.b), tol=1e-10, maxit=5000)
            assert res["code"] == cg.CG_OK
            out.setdefault(exchange, []).append((host(x), res["iterations"]))
        s.set_opts(exchange=2, small_path=1)     # the mode overrides the LDS path
        x, res = s.solve(dev(p.b), tol=1e-10, maxit=5000)
        out[2].append((host(x), res["iterations"]))
    ref_x, ref_it = out[0][0]
    for runs in out.values():
        for xk, it in runs:
            assert it == ref_it and np.array_equal(xk, ref_x)


def test_shared_p_modes_reject_unsupported_combinations(cg):
    p = I.poisson2d_problem(16)
    with cg.Solver(p.A) as s:
        for exchange in (2, 3):   # rejected whether or not managed memory is supported
            with pytest.raises(cg.CgError):
                s.set_opts(exchange=exchange, precision=cg.PREC_MIXED)
            with pytest.raises(cg.CgError):
                s.set_opts(exchange=exchange, precond=cg.PC_FSAI)
        with pytest.raises(cg.CgError):
            s.set_opts(exchange=4)
        # a rejected option leaves the handle as it was
        x, res = s.solve(dev(p.b), tol=1e-10)
        assert res["code"] == cg.CG_OK


def test_split_spmv_matches_oracle(cg):
    A = I.random_spd_lognormal(5000, seed=8)
    x = np.random.default_rng(1).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    for rb, re in [(0, 0), (0, 2500), (1000, 4000)]:
        with cg.Solver(A, rb, re) as s:
            y = host(s.spmv(dev(x)))
        assert spmv_err(A, x, y, ref) <= 1e-12


def test_automatic_stream_tiles_for_large_irregular_matrices(cg):
    """A matrix of irregular short rows (mean 21, longest 123: slices would
    pad 3.6x) with n >= 131,072 takes stream tiles automatically, whose SpMV
    is bit-exact against the oracle (rows summed in CSR order); the same law
    at 100,000 rows keeps the vector bins (rows reduced across lanes: within
    the rounding bar).  Fixed-work CG tracks the oracle's in both."""
    for n, want in ((140_000, 2), (100_000, 1)):
        A = I.random_spd_lognormal(n, 4, mean_degree=10.0, max_degree=100)
        x = np.random.default_rng(6).uniform(-1, 1, A.n)
        b = A.scipy() @ np.ones(A.n)
        with cg.Solver(A) as s:
            assert used_kind(s, A.n) == want
            y, ref_y = host(s.spmv(dev(x))), oracle.spmv(A, x)
            assert spmv_err(A, x, y, ref_y) <= 1e-12
            if want == 2:
                assert np.array_equal(y, ref_y)
            xs, res = s.solve(dev(b), tol=0.0, maxit=15)
        ref = oracle.cg(A, b, tol=0.0, maxit=15)
        assert res["iterations"] == 15
        # bar: 4x the distance between the oracle and a second correct float64
        # CG (scipy products, BLAS dots)
        S = A.scipy()
        xa, r, rho = np.zeros(A.n), b.copy(), b @ b
        pa = r.copy()
        for _ in range(15):
            qv = S @ pa
            alpha = rho / (pa @ qv)
            xa += alpha * pa
            r -= alpha * qv
            rho, rho_old = r @ r, rho
            pa = r + (rho / rho_old) * pa
        nx = np.linalg.norm(ref["x"])
        spread = np.linalg.norm(xa - ref["x"]) / nx
        assert np.linalg.norm(host(xs) - ref["x"]) / nx <= max(1e-13, 4 * spread), spread


@pytest.mark.parametrize("rb,re", [(0, 1001), (37, 990), (64, 700), (1000, 1001)])
def test_split_gap_coded_slices(cg, rb, re):
    """Gap-coded slices on a GPU block that starts inside the matrix (their
    first-column offsets count from global row indices): the split SpMV is
    bit-exact against the oracle, and fixed-work CG iterates equal those of
    plain slices on the same split bit for bit (same rows, same summation
    and partial order)."""
    A = SPMV_CASES["poisson3d_ragged"]()
    assert A.n == 1001 and gaps_apply(A)
    x = np.random.default_rng(5).uniform(-1, 1, A.n)
    b = I.rhs_of(A, I.uniform_vector(A.n, [5, 1]))
    ref = oracle.spmv(A, x)
    out = {}
    for kind in (3, 7):
        with cg.Solver(A, rb, re) as s:
            s.set_opts(spmv_kind=kind, small_path=0, host_threads=2)
            assert np.array_equal(host(s.spmv(dev(x))), ref)
            xs, res = s.solve(dev(b), tol=0.0, maxit=20)
            assert res["spmv_kind"] == kind and res["iterations"] == 20
            out[kind] = host(xs)
    assert np.array_equal(out[3], out[7])


@pytest.mark.parametrize("small_path", [1, 0])
def test_cg_edge_cases(cg, small_path):
    p = I.poisson2d_problem(16)
    n = p.A.n
    with cg.Solver(p.A) as s:
        s.set_opts(small_path=small_path)
        # b = 0: x = 0 whatever the initial guess
        x, res = s.solve(dev(np.zeros(n)), dev(np.ones(n)))
        assert res["code"] == cg.CG_OK and not host(x).any()
        # maxit = 0 leaves x untouched
        x0 = np.linspace(-1, 1, n)
        x, res = s.solve(dev(p.b), dev(x0), maxit=0)
        assert res["code"] == cg.CG_MAXIT and np.array_equal(host(x), x0)
        # exact initial guess: converged with no iteration
        x, res = s.solve(dev(p.b), dev(p.xstar.copy()), tol=1e-8)
        assert res["code"] == cg.CG_OK and res["iterations"] == 0
        # NaN in b: breakdown
        b = p.b.copy(); b[5] = np.nan
        x, res = s.solve(dev(b), maxit=10)
        assert res["code"] == cg.CG_EBREAKDOWN
    B = I.poisson2d(16)
    B.val = np.where(B.col == np.repeat(np.arange(n), np.diff(B.row_ptr)), -4.0, B.val)
    with cg.Solver(B) as s:
        s.set_opts(small_path=small_path)
        x, res = s.solve(dev(np.ones(n)), maxit=100)
        assert res["code"] == cg.CG_EBREAKDOWN


@pytest.mark.parametrize("n", [4998, (1 << 21) + 4])
@pytest.mark.parametrize("case", ["odd_step", "even_step"])
def test_breakdown_keeps_x_of_the_last_full_iteration(cg, case, n):
    """Indefinite block-diagonal systems whose p^T q turns non-positive at
    iteration 1 (odd) or 2 (even): x holds every update before the breakdown
    (with x updated every other iteration, the odd case flushes the owed
    term), as the oracle's run.  n = 2^21 + 4 fills the vector kernels' whole
    grid several times over, so workgroups that start after workgroup 0 has
    recorded the breakdown must still add their share of the owed term."""
    dv, bv = ([1.0, -1.0], [1.0, 0.5]) if case == "odd_step" else ([1.0, 3.0, -1.0], [1.0, 1.0, 0.05])
    reps = n // len(dv)
    d, b = np.tile(dv, reps), np.tile(bv, reps)
    A = I.CSR(d.size, np.arange(d.size + 1, dtype=np.int32), np.arange(d.size, dtype=np.int32), d)
    ref = oracle.cg(A, b, tol=1e-12, maxit=100)
    assert ref["status"] == cg.CG_EBREAKDOWN and ref["iterations"] == (1 if case == "odd_step" else 2)
    xs = []
    for fuse in (cg.FUSE_ON, cg.FUSE_OFF):
        with cg.Solver(A) as s:
            s.set_opts(small_path=0, fuse_dir=fuse, spmv_kind=6)
            x, res = s.solve(dev(b), tol=1e-12, maxit=100)
        assert res["code"] == cg.CG_EBREAKDOWN and res["iterations"] == ref["iterations"]
        assert res["fused_dir"] == (fuse == cg.FUSE_ON) and res["spmv_kind"] == 6
        xs.append(host(x))
    # alpha and beta come from dot products over n entries summed in other
    # orders (relative error within n u each); a missing owed term would
    # be off by alpha p, of the order of x itself
    u = 2.0 ** -53
    assert np.abs(xs[0] - ref["x"]).max() <= 4 * n * u * np.abs(ref["x"]).max()
    # the direction update inside the SpMV flushes the owed term as the
    # separate kernel does
    assert np.array_equal(xs[0], xs[1])


def test_deterministic_across_solves(cg):
    p = I.random_spd_problem(20000, seed=5)
    with cg.Solver(p.A) as s:
        x1, r1 = s.solve(dev(p.b), tol=1e-10)
        x2, r2 = s.solve(dev(p.b), tol=1e-10)
    assert r1["iterations"] == r2["iterations"] and torch.equal(x1, x2)


@pytest.mark.parametrize("n", [1, 2, 1001, 1 << 20])
@pytest.mark.parametrize("offset", [0, 1])
def test_hbm_copy(cg, n, offset):
    """The library's streaming copy: exact for any length and alignment
    (offset 1: neither pointer 16-byte aligned)."""
    src = torch.rand(n + offset, dtype=torch.float64, device="cuda")[offset:]
    dst = torch.full((n + offset,), -1.0, dtype=torch.float64, device="cuda")[offset:]
    cg.hbm_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("n", [0, 1, 7, 1001, 1 << 20])
@pytest.mark.parametrize("offset", [0, 1])
def test_gather_reference(cg, n, offset):
    """The library's random gather: dst = src[idx] exactly, any length and
    alignment (offset 1: idx and dst not 16-byte aligned)."""
    src = torch.rand(300_000, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(n + offset)
    idx = torch.randint(0, src.numel(), (n + offset,), dtype=torch.int32, device="cuda", generator=g)[offset:]
    dst = torch.full((n + offset,), -1.0, dtype=torch.float64, device="cuda")[offset:]
    cg.gather(src, idx, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst, src[idx.long()])


@pytest.mark.parametrize("fuse", [1, 2])   # cg.FUSE_ON, cg.FUSE_OFF
@pytest.mark.parametrize("stride", [1, 7])
def test_spmv_event_sampling(cg, stride, fuse):
    """cg_opts.profile = P times the SpMV of iterations 0, P, 2P, ...: the
    count follows, the mean is positive, and the iterates are unchanged
    (with the direction update inside the SpMV too, where the launch that
    ends the last iteration runs no SpMV and is not counted)."""
    p = I.poisson3d_problem(24)
    b = dev(p.b)
    with cg.Solver(p.A) as s:
        s.set_opts(small_path=0, fuse_dir=fuse)
        x0, r0 = s.solve(b, tol=0.0, maxit=50)
        s.set_opts(profile=stride, small_path=0)
        x1, r1 = s.solve(b, tol=0.0, maxit=50)
        # a solve that converges: only SpMVs of iterations that ran
        s.set_opts(profile=1, small_path=0)
        x2, r2 = s.solve(b, tol=1e-8, maxit=10_000)
    assert r1["fused_dir"] == (fuse == cg.FUSE_ON)
    assert r0["n_spmv"] == 0 and r1["n_spmv"] == (50 + stride - 1) // stride
    assert r1["t_spmv"] > 0.0
    assert torch.equal(x0, x1)
    assert r2["converged"] == 1 and r2["n_spmv"] == r2["iterations"]


FUSED_CASES = {
    "poisson3d_24": lambda: I.poisson3d_problem(24),          # n even, 216 slices
    "poisson2d_61": lambda: I.poisson2d_problem(61, seed=3),  # n odd: a last lane with one row
    "poisson3d_65": lambda: I.poisson3d_problem(65, seed=4),  # n odd, 4,291 slices over the whole grid
}


@pytest.mark.parametrize("n", [2, 3, 65, 130, 191])
def test_fused_direction_update_tiny_chains(cg, n):
    """The fused direction update on chains of 2 to 191 rows (one slice, a
    slice pair with one slice, odd tails): bitwise the separate kernels, and
    the solution within the CG bar of a dense solve."""
    A = I.poisson2d(n, 1)
    b = np.random.default_rng(n).uniform(-1, 1, n)
    out = []
    for fuse in (cg.FUSE_OFF, cg.FUSE_ON):
        with cg.Solver(A) as s:
            s.set_opts(small_path=0, fuse_dir=fuse, spmv_kind=6)
            x, r = s.solve(dev(b), tol=1e-12, maxit=1000)
        out.append((host(x), r))
    (x0, r0), (x1, r1) = out
    assert r1["fused_dir"] == 1 and r0["fused_dir"] == 0 and r1["spmv_kind"] == 6
    assert r0["iterations"] == r1["iterations"] and np.array_equal(x0, x1)
    xd = np.linalg.solve(A.scipy().toarray(), b)
    assert np.linalg.norm(x1 - xd) <= 2 * 2.0 * 1e-12 * np.linalg.norm(xd) * 3   # kappa(A) < 3


@pytest.mark.parametrize("maxit,tol,every", [(1, 0.0, 32), (2, 0.0, 1), (3, 0.0, 2), (57, 0.0, 5),
                                             (20000, 1e-10, 32)])
@pytest.mark.parametrize("name", list(FUSED_CASES))
def test_fused_direction_update_is_bitwise(cg, name, maxit, tol, every):
    """cg_opts.fuse_dir: the end of iteration k (beta, the stop test,
    p_{k+1}, the x terms owed every other iteration) inside the SpMV of
    iteration k+1 gives bitwise the x, iteration count and residuals of the
    separate kernels: stops at odd and even iterations, by the iteration
    limit and by the tolerance, with polls after every iteration, every
    other and every 5th.  The run is the oracle's within the CG bar."""
    p = FUSED_CASES[name]()
    out = []
    for fuse in (cg.FUSE_OFF, cg.FUSE_ON):
        with cg.Solver(p.A) as s:
            s.set_opts(small_path=0, fuse_dir=fuse, check_every=every)
            x, r = s.solve(dev(p.b), tol=tol, maxit=maxit)
        out.append((host(x), r))
    (x0, r0), (x1, r1) = out
    print(f"[fused] {name} maxit={maxit} it={r1['iterations']} kind={r1['spmv_kind']}", flush=True)
    assert r0["fused_dir"] == 0 and r1["fused_dir"] == 1 and r1["spmv_kind"] == 6
    assert r0["code"] == r1["code"] and r0["iterations"] == r1["iterations"]
    assert r0["rel_res_recur"] == r1["rel_res_recur"] and r0["rel_res_true"] == r1["rel_res_true"]
    assert np.array_equal(x0, x1)
    if maxit <= 3:
        ref = oracle.cg(p.A, p.b, tol=0.0, maxit=maxit)
        assert np.linalg.norm(x1 - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-13


def test_full_size_poisson3d_256(cg):
    """Full 256^3 size in the benchmark's launch configuration: SpMV against
    the oracle on every row; a fixed-work solve checked by properties that
    hold at any size (recomputed true residual, first iterates)."""
    p = I.poisson3d_problem(256)
    A = p.A
    print(f"[full] poisson3d 256^3 n={A.n} nnz={A.nnz}", flush=True)
    x = np.random.default_rng(2).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    from paper_2608_09647_amd import autotune
    with cg.Solver(A) as s:
        sched = autotune.spmv_schedule(s, A, dev(p.b), tune_if_missing=False)
        print(f"[full] schedule {sched}", flush=True)
        s.set_opts(profile=1)
        y = host(s.spmv(dev(x)))
        assert used_kind(s, A.n) == 6
        # stencil slices sum every row in the oracle's order: equal bits
        assert np.array_equal(y, ref)
        del y, ref
        xg, res = s.solve(dev(p.b), tol=0.0, maxit=3)
        x3 = host(xg)
        xg, res500 = s.solve(dev(p.b), tol=0.0, maxit=500)
        x500 = host(xg)
    ora3 = oracle.cg(A, p.b, tol=0.0, maxit=3)
    assert np.linalg.norm(x3 - ora3["x"]) / np.linalg.norm(ora3["x"]) <= 1e-13
    assert res500["iterations"] == 500 and res500["n_spmv"] == 500
    true = np.linalg.norm(p.b - oracle.spmv(A, x500)) / np.linalg.norm(p.b)
    assert abs(res500["rel_res_true"] - true) <= 1e-6 * true
    assert true < 1e-2   # 500 CG steps on the 7-point Laplacian reduce the residual well below 1


# ----------------------------------------------------------------------------- mixed precision

@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4, 5, 7])
@pytest.mark.parametrize("name", ["poisson3d_ragged", "random_spd_30k", "diffusion_100"])
def test_spmv_f32_matches_oracle(cg, name, kind):
    A = SPMV_CASES[name]()
    x32 = np.random.default_rng(4).uniform(-1, 1, A.n).astype(np.float32)
    ref = oracle.spmv_f32(A, x32)
    with cg.Solver(A) as s:
        s.set_opts(precision=cg.PREC_MIXED, spmv_kind=kind)
        y = host(s.spmv_f32(torch.from_numpy(x32).cuda()))
        used = used_kind(s, A.n)
    absA = sp.csr_matrix((np.abs(A.val.astype(np.float32)), A.col, A.row_ptr), shape=(A.n, A.n))
    scale = absA @ np.abs(x32).astype(np.float64) + 1e-30
    L = int(np.diff(A.row_ptr).max())
    assert np.max(np.abs(y.astype(np.float64) - ref) / scale) <= 2 * L * 2.0 ** -24
    if used in (2, 3, 4, 7):
        # stream and sliced rows are summed in float32 left to right: the oracle's order
        assert np.array_equal(y, ref)


MIXED_CASES = {
    "random_spd_20k": lambda: I.random_spd_problem(20000, seed=3),
    "poisson3d_32": lambda: I.poisson3d_problem(32),
    "diffusion_64": lambda: I.diffusion_problem(64, seed=10_000),
}


@pytest.mark.parametrize("name", list(MIXED_CASES))
def test_mixed_precision_matches_oracle(cg, name):
    p = MIXED_CASES[name]()
    print(f"[mixed] {name} n={p.A.n}", flush=True)
    ref = oracle.cg_mixed(p.A, p.b, tol=1e-10, maxit=20000)
    ref64 = oracle.cg(p.A, p.b, tol=1e-10, maxit=20000)
    with cg.Solver(p.A) as s:
        s.set_opts(precision=cg.PREC_MIXED)
        x, res = s.solve(dev(p.b), tol=1e-10, maxit=20000)
    x = host(x)
    assert res["code"] == cg.CG_OK and ref["status"] == oracle.OK
    # success is decided on the float64 true residual, recomputed here by the oracle
    true = np.linalg.norm(p.b - oracle.spmv(p.A, x)) / np.linalg.norm(p.b)
    assert true < 1e-10
    assert res["fp64_residuals"] >= 2 and not res["fell_back"]
    assert abs(res["iterations"] - ref["iterations"]) <= max(3, 0.1 * ref["iterations"])
    kappa = kappa_of(name, p.A)
    err = np.linalg.norm(x - ref64["x"]) / np.linalg.norm(ref64["x"])
    print(f"[mixed] {name}: {res['iterations']} float32 iterations ({ref['iterations']} oracle), "
          f"{res['fp64_residuals']} float64 residuals, error vs float64 solution {err:.2e}", flush=True)
    assert err <= 2 * kappa * 1e-10


def test_mixed_precision_edge_cases(cg):
    p = I.poisson2d_problem(16)
    n = p.A.n
    with cg.Solver(p.A) as s:
        s.set_opts(precision=cg.PREC_MIXED)
        x, res = s.solve(dev(np.zeros(n)), dev(np.ones(n)))
        assert res["code"] == cg.CG_OK and not host(x).any()
        x, res = s.solve(dev(p.b), dev(p.xstar.copy()), tol=1e-8)
        assert res["code"] == cg.CG_OK and res["iterations"] == 0
        x, res = s.solve(dev(p.b), maxit=3)
        assert res["code"] == cg.CG_MAXIT and res["iterations"] == 3
    with cg.Solver(p.A, 0, n // 2) as s:
        with pytest.raises(cg.CgError):
            s.set_opts(precision=cg.PREC_MIXED)


def test_matrix_market_file_solves_like_the_generated_matrix(cg, tmp_path):
    """A Poisson system written as a symmetric Matrix Market file (lower
    triangle), read back by the library and solved on the GPU: the same CSR
    as the generator's, and the oracle's CG result."""
    import scipy.io
    p = I.poisson3d_problem(20)
    path = str(tmp_path / "poisson.mtx")
    scipy.io.mmwrite(path, sp.tril(p.A.scipy(), format="coo"), symmetry="symmetric", precision=17)
    A, info = cg.read_matrix_market(path)
    assert info["symmetric"] and np.array_equal(A.row_ptr, p.A.row_ptr)
    assert np.array_equal(A.col, p.A.col) and np.array_equal(A.val, p.A.val)
    ref = oracle.cg(p.A, p.b, tol=1e-10, maxit=5000)
    with cg.Solver(A) as s:
        x, res = s.solve(dev(p.b), tol=1e-10, maxit=5000)
    lam = 2 - 2 * np.cos(np.arange(1, 21) * np.pi / 21)
    check_cg(p.A, p.b, host(x), res, ref, 1e-10, 3 * lam.max() / (3 * lam.min()))


def test_paper_inputs_absolute_tolerance(cg):
    """Algorithm 1's own inputs: b = 1, x0 = 0, stop when sqrt(rho) < tau with
    tau and I_max from tests/golden/paper_constants.json.  The absolute test
    is the relative one at tol = tau / ||b||."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")) as f:
        g = json.load(f)["algorithm1_defaults"]
    A = I.poisson3d(24)
    b = np.ones(A.n)
    tol = g["tau"] / np.linalg.norm(b)
    ref = oracle.cg(A, b, tol=tol, maxit=g["i_max"])
    with cg.Solver(A) as s:
        x, res = s.solve(dev(b), tol=tol, maxit=g["i_max"])
    assert res["code"] == cg.CG_OK and ref["status"] == oracle.OK
    assert res["rel_res_recur"] * np.linalg.norm(b) < g["tau"]          # sqrt(rho) < tau
    assert abs(res["iterations"] - ref["iterations"]) <= max(2, 0.05 * ref["iterations"])
    lam = 2 - 2 * np.cos(np.arange(1, 25) * np.pi / 25)
    assert np.linalg.norm(host(x) - ref["x"]) / np.linalg.norm(ref["x"]) <= 2 * (lam.max() / lam.min()) * tol * 10



@pytest.mark.parametrize("name", ["poisson3d_ragged", "diffusion_100", "poisson2d_64", "poisson3d_planes_256"])
def test_sliced_pairs_track_stencil_pairs_bitwise(cg, name):
    """Plain slices with two rows per lane (columns streamed, a length byte per
    row), the same with gap-coded columns, and stencil slices with two rows
    per lane sum every row in CSR order and walk the same slice pairs with the
    same grid, so p^T q is added in the same order: fixed-work CG iterates are
    equal bit for bit."""
    A = SPMV_CASES[name]()
    b = I.rhs_of(A, I.uniform_vector(A.n, [17, 1]))
    out = {}
    for kind in (3, 6, 7):
        with cg.Solver(A) as s:
            s.set_opts(spmv_kind=kind, small_path=0)
            xs, res = s.solve(dev(b), tol=0.0, maxit=31)
            out[kind] = (res["spmv_kind"], host(xs))
    assert out[3][0] == 3 and out[6][0] == 6 and out[7][0] == 7
    assert np.array_equal(out[3][1], out[6][1])
    assert np.array_equal(out[7][1], out[6][1])


def _csr_from_lists(n, rows):
    """CSR of per-row (columns, values) lists, columns kept in the given order."""
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(c) for c, _ in rows])
    ci = np.concatenate([np.asarray(c, np.int32) for c, _ in rows])
    va = np.concatenate([np.asarray(v, np.float64) for _, v in rows])
    return I.CSR(n, rp, ci, va)


@pytest.mark.parametrize("case", ["gap_65536", "gap_65537", "first_524287", "first_524288",
                                  "first_-524288", "first_-524289", "eight_per_row", "wide_rows",
                                  "odd_rows"])
def test_gap_coded_slices_edges(cg, case):
    """Gap-coded slices at the edge of their range: a gap of 65,536 (the
    largest one coded) and of 65,537 (plain slices); a row's first column
    2^19 - 1 and -2^19 from its own index (coded) and one further (plain
    slices); rows of 8 entries (coded) and of 9 (plain slices); and an odd
    row count with empty rows (the last pair holds one slice, empty rows
    start at the last row).  The SpMV is bit-exact against the oracle in
    every case."""
    rng = np.random.default_rng(21)
    if case.startswith(("gap_", "first_")):
        kind, far = case.split("_")
        far = int(far)
        n = 70_000 if kind == "gap" else 600_000
        rows = []
        for i in range(n):
            cols = sorted({i, max(0, i - 1), min(n - 1, i + 1)})
            rows.append((cols, rng.uniform(-1, 1, len(cols))))
        if kind == "gap":
            rows[3] = ([3, 3 + far], [4.0, -0.5])    # row 3's gap
        else:
            r = 7 if far > 0 else 7 - far            # a row whose only column is r + far
            rows[r] = ([r + far], [4.0])
        expect = 7 if case in ("gap_65536", "first_524287", "first_-524288") else 3
    elif case == "eight_per_row":
        n = 5000        # every row at the paired tiles' full width, 8 entries
        rows = [(sorted(rng.choice(n, 8, replace=False)), rng.uniform(-1, 1, 8)) for _ in range(n)]
        expect = 7
    elif case == "wide_rows":
        n = 3000
        rows = [(sorted(rng.choice(n, 9, replace=False)), rng.uniform(-1, 1, 9)) for _ in range(n)]
        expect = 3
    else:
        n = 64 * 5 + 37
        rows = []
        for i in range(n):
            if i % 7 == 3:
                rows.append(([], []))
            else:
                cols = sorted(set(rng.choice(n, 4, replace=False)) | {i})
                rows.append((cols, rng.uniform(-1, 1, len(cols))))
        expect = 7
    A = _csr_from_lists(n, rows)
    assert gaps_apply(A) == (expect == 7)
    x = rng.uniform(-1, 1, n)
    ref = oracle.spmv(A, x)
    with cg.Solver(A) as s:
        s.set_opts(spmv_kind=7, small_path=0)
        assert used_kind(s, n) == expect
        assert np.array_equal(host(s.spmv(dev(x))), ref)


@pytest.mark.parametrize("name", ["poisson3d_24", "poisson3d_ragged", "poisson2d_64", "diffusion_100"])
def test_stencil_slices_chosen_and_exact(cg, name):
    """Stencil matrices take stencil slices automatically; SpMV bit-exact
    (rows summed in CSR order) and a fixed-work CG that tracks the dictionary
    tiling's (the p^T q partials may be added in another order)."""
    A = SPMV_CASES[name]()
    assert stencil_applies(A)
    x = np.random.default_rng(13).uniform(-1, 1, A.n)
    b = I.rhs_of(A, I.uniform_vector(A.n, [13, 1]))
    out = {}
    for kind in (0, 4):
        with cg.Solver(A) as s:
            s.set_opts(spmv_kind=kind, small_path=0)
            y = host(s.spmv(dev(x)))
            used = used_kind(s, A.n)
            xs, res = s.solve(dev(b), tol=0.0, maxit=25)
            out[kind] = (used, y, host(xs))
    assert out[0][0] == 6 and out[4][0] == 4
    assert np.array_equal(out[0][1], oracle.spmv(A, x))
    assert np.array_equal(out[0][1], out[4][1])
    # both fixed-work iterates within 4x the distance between the oracle and a
    # second correct float64 CG (the high-contrast field amplifies the order
    # in which p^T q is summed)
    fixed = oracle.cg(A, b, tol=0.0, maxit=25)
    S = A.scipy()
    xa, r, rho = np.zeros(A.n), b.copy(), b @ b
    pa = r.copy()
    for _ in range(25):
        qv = S @ pa
        alpha = rho / (pa @ qv)
        xa += alpha * pa
        r -= alpha * qv
        rho, rho_old = r @ r, rho
        pa = r + (rho / rho_old) * pa
    nx = np.linalg.norm(fixed["x"])
    bar = max(1e-12, 4 * np.linalg.norm(xa - fixed["x"]) / nx)
    for kind in (0, 4):
        assert np.linalg.norm(out[kind][2] - fixed["x"]) / nx <= bar, kind


def test_stencil_slices_fall_back_on_many_offsets(cg):
    """A slice with more than 8 distinct column offsets (rows of <= 8 entries)
    is not stencil-sliced: kind 6 falls back to the dictionary tiles."""
    n = 1024
    rng = np.random.default_rng(4)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for _ in range(3):
        perm = rng.permutation(n)
        a, b2 = perm[0::2], perm[1::2]
        rows += [a, b2]
        cols += [b2, a]
    r, cidx = np.concatenate(rows), np.concatenate(cols)
    S = sp.csr_matrix((np.where(r == cidx, 8.0, -0.5), (r, cidx)), shape=(n, n))
    S.sum_duplicates()
    S.sort_indices()
    A = I.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    assert np.diff(A.row_ptr).max() <= 8 and not stencil_applies(A)
    x = rng.uniform(-1, 1, n)
    with cg.Solver(A) as s:
        s.set_opts(spmv_kind=6)
        assert used_kind(s, n) in (3, 4)
        assert np.array_equal(host(s.spmv(dev(x))), oracle.spmv(A, x))



@pytest.mark.parametrize("shape", [(13, 11, 7), (9, 9, 9), (64, 2, 1), (65, 1, 1), (5, 5, 5), (8, 8, 3), (12, 12, 1)])
def test_stencil_two_rows_per_lane_edges(cg, shape):
    """Odd row counts (the last row alone, in the SpMV and in the x/p update
    that works on pairs of entries), odd slice counts (a pair with one slice)
    and single-slice systems: SpMV bit-exact, dot product and a multi-kernel
    solve against the oracle."""
    A = I.poisson3d(*shape)
    assert stencil_applies(A)
    x = np.random.default_rng(17).uniform(-1, 1, A.n)
    b = I.rhs_of(A, I.uniform_vector(A.n, [17, 1]))
    ref = oracle.cg(A, b, tol=1e-10, maxit=5000)
    with cg.Solver(A) as s:
        s.set_opts(small_path=0, spmv_kind=6)    # requested: tiny systems may not pass the padding rule
        assert used_kind(s, A.n) == 6
        assert np.array_equal(host(s.spmv(dev(x))), oracle.spmv(A, x))
        xs, res = s.solve(dev(b), tol=1e-10, maxit=5000)
    assert res["code"] == cg.CG_OK
    assert abs(res["iterations"] - ref["iterations"]) <= max(2, 0.05 * ref["iterations"])
    assert np.linalg.norm(b - oracle.spmv(A, host(xs))) / np.linalg.norm(b) <= 1.01e-10


def test_stencil_misaligned_output_uses_one_row_per_lane(cg):
    """An output vector that is not 16-byte aligned takes the one-row-per-lane
    kernel; the result is the same bits."""
    A = I.poisson3d(10)
    x = np.random.default_rng(19).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, x)
    with cg.Solver(A) as s:
        ybuf = torch.zeros(A.n + 1, dtype=torch.float64, device="cuda")
        y_odd = ybuf[1:]                         # 8 bytes past a 16-byte boundary
        s.spmv(dev(x), y_odd)
        assert np.array_equal(host(y_odd), ref)
        assert np.array_equal(host(s.spmv(dev(x))), ref)


@pytest.mark.parametrize("case", ["small_path", "multi_kernel", "split"])
def test_host_vectors_match_device_vectors(cg, case):
    """cg_opts.vectors = CG_VECTORS_HOST: b, x and y are host arrays, staged
    through the library's own device buffers; results equal the device-pointer
    calls bit for bit."""
    p = I.poisson2d_problem(48) if case == "small_path" else I.poisson3d_problem(24)
    n = p.A.n
    rb, re = (0, n // 2) if case == "split" else (0, n)
    x_in = np.random.default_rng(21).uniform(-1, 1, n)
    with cg.Solver(p.A, rb, re) as s:
        s.set_opts(host_threads=3)
        y_dev = host(s.spmv(dev(x_in)))
        x_dev, r_dev = s.solve(dev(p.b), tol=1e-10, maxit=5000)
        x_dev = host(x_dev)
        s.set_opts(vectors=cg.VECTORS_HOST, host_threads=3)
        y_host = s.spmv_host(x_in)
        x0 = np.zeros(n)
        x_host, r_host = s.solve_host(p.b, x0, tol=1e-10, maxit=5000)
        # a rejected use: the allocation-free solve takes device vectors only
        if case != "split":
            _, rn = s.solve_noalloc(dev(p.b), torch.zeros(n, dtype=torch.float64, device="cuda"), check=False)
            assert rn["code"] == cg.CG_EINVAL
    assert x_host is x0
    assert np.array_equal(y_host, y_dev) and np.array_equal(x_host, x_dev)
    assert r_host["code"] == r_dev["code"] == cg.CG_OK and r_host["iterations"] == r_dev["iterations"]
    assert r_host["rel_res_true"] == r_dev["rel_res_true"]


def test_small_path_launch_is_event_timed(cg):
    """cg_opts.profile on the single-workgroup path: an event pair around the
    one launch gives t_spmv (n_spmv = 1), within the host-timed t_gpu; the
    solution is bitwise the one of the unprofiled solve."""
    p = I.poisson2d_problem(64, seed=1)
    with cg.Solver(p.A) as s:
        s.set_opts(small_path=1)
        x0, r0 = s.solve(dev(p.b), tol=1e-10, maxit=20000)
        assert r0["n_spmv"] == 0 and r0["t_spmv"] == 0.0
        s.set_opts(profile=1)
        x1, r1 = s.solve(dev(p.b), tol=1e-10, maxit=20000)
    assert r1["n_spmv"] == 1 and 0.0 < r1["t_spmv"] <= r1["t_gpu"]
    assert r1["iterations"] == r0["iterations"] and np.array_equal(host(x0), host(x1))
