"""Pins for the CPU oracle's SpMV, CG, PCG and mixed-precision CG.

Each test checks the oracle against something other than itself: dense linear
algebra, exact integer arithmetic, closed-form eigenvalues, theorems about CG
in exact arithmetic that survive rounding on well-conditioned problems, or a
hand-computed first step.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2608_09647_amd import inputs as I

EPS = np.finfo(np.float64).eps


def csr_from_dense(M):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return I.CSR(M.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


def random_spd_dense(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T, lam


# ----------------------------------------------------------------------------- SpMV

def test_spmv_matches_dense_within_sum_order_bound():
    rng = np.random.default_rng(0)
    n = 64
    M = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.2)
    M[5, :] = 0.0                        # an empty row
    M[7, :] = rng.standard_normal(n)     # a full row
    A = csr_from_dense(M)
    x = rng.standard_normal(n)
    y = oracle.spmv(A, x)
    ref = M @ x
    L = int(np.diff(A.row_ptr).max())
    bound = 2 * L * EPS * (np.abs(M) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(y - ref) <= bound)
    assert y[5] == 0.0


def test_spmv_integer_inputs_are_exact():
    A = I.poisson3d(8)
    rng = np.random.default_rng(1)
    xi = rng.integers(-1000, 1001, size=A.n)
    S = sp.csr_matrix((A.val.astype(np.int64), A.col, A.row_ptr), shape=(A.n, A.n))
    exact = (S @ xi).astype(np.float64)
    y = oracle.spmv(A, xi.astype(np.float64))
    assert np.array_equal(y, exact)


def test_spmv_ones_counts_missing_neighbours():
    # Dirichlet Laplacian: (A 1)_i = number of grid neighbours outside the domain.
    nx = 9
    A = I.poisson2d(nx)
    y = oracle.spmv(A, np.ones(A.n))
    ix, iy = np.arange(A.n) % nx, np.arange(A.n) // nx
    missing = (ix == 0).astype(int) + (ix == nx - 1) + (iy == 0) + (iy == nx - 1)
    assert np.array_equal(y, missing.astype(np.float64))


def test_spmv_random_spd_row_sums_equal_shift():
    A = I.random_spd_lognormal(3000, seed=7)
    y = oracle.spmv(A, np.ones(A.n))
    absrow = np.add.reduceat(np.abs(A.val), A.row_ptr[:-1])
    np.testing.assert_allclose(y, 0.01, atol=8 * EPS * absrow.max())


def test_spmv_thread_count_does_not_change_bits():
    A = I.random_spd_lognormal(5000, seed=11)
    x = np.random.default_rng(2).standard_normal(A.n)
    t0 = oracle.max_threads()
    oracle.set_threads(1)
    y1 = oracle.spmv(A, x)
    oracle.set_threads(max(2, t0))
    y2 = oracle.spmv(A, x)
    oracle.set_threads(t0)
    assert np.array_equal(y1, y2)


# float32 SpMV (the inner product of the mixed-precision solve).  Each pin is
# also run against a copy of the routine with a planted slip, which it must
# reject, so the pin is known to see that kind of mistake.

U32 = 2.0 ** -24    # unit roundoff of float32


def _spmv_f32_f64_accumulator(A, x32):
    """Planted slip: float32 operands, but products and sums in float64."""
    v = A.val.astype(np.float32).astype(np.float64)
    x = np.asarray(x32, dtype=np.float32).astype(np.float64)
    y = np.empty(A.n, dtype=np.float32)
    for i in range(A.n):
        s = 0.0
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            s += v[k] * x[A.col[k]]
        y[i] = np.float32(s)
    return y


def _f32_rounding_rows():
    """Two rows whose float32 results follow by hand from IEEE rounding.
    Row 0: 1 + 2^-24 + 2^-24 with x = 1; in float32 each 2^-24 is half an
    ulp of 1 and is lost (ties to even), so the sum is 1; summed in float64
    and rounded at the end it would be 1 + 2^-23.
    Row 1: -(1 + 2^-11) * 1 + (1 + 2^-12)^2; the exact second product
    1 + 2^-11 + 2^-24 rounds (tie, to even) to 1 + 2^-11 in float32, so the
    row is exactly 0; with a float64 (or fused) product the 2^-24 survives."""
    a = 1.0 + 2.0 ** -12                            # exact in float32
    x = np.array([1.0, a, 1.0, 1.0], dtype=np.float32)
    rp = np.array([0, 3, 5, 5, 5], dtype=np.int32)
    ci = np.array([0, 2, 3, 0, 1], dtype=np.int32)
    val = np.array([1.0, U32, U32, -(1.0 + 2.0 ** -11), a])
    A = I.CSR(4, rp, ci, val)
    return A, x, np.array([1.0, 0.0, 0.0, 0.0], dtype=np.float32)


def test_spmv_f32_rounds_every_product_and_sum_in_float32():
    A, x, want = _f32_rounding_rows()
    assert np.array_equal(oracle.spmv_f32(A, x), want)
    assert oracle.spmv_f32(A, x).dtype == np.float32
    assert not np.array_equal(_spmv_f32_f64_accumulator(A, x), want)


def test_spmv_f32_integer_inputs_are_exact():
    """Poisson 6/-1 with integer x in [-1000, 1000]: every partial sum is an
    integer below 2^24, exact in float32 in any order."""
    A = I.poisson3d(8)
    xi = np.random.default_rng(4).integers(-1000, 1001, size=A.n)
    S = sp.csr_matrix((A.val.astype(np.int64), A.col, A.row_ptr), shape=(A.n, A.n))
    exact = (S @ xi).astype(np.float32)
    assert np.array_equal(oracle.spmv_f32(A, xi.astype(np.float32)), exact)


def test_spmv_f32_within_float32_sum_order_bound():
    """Against a float64 dense matvec of the float32-rounded operands: the
    error of a row of L rounded products summed in float32 is at most
    gamma_L = L u / (1 - L u) times sum |a_ik x_k| (u = 2^-24); and it is far
    above float64's, so a float64 accumulator would show."""
    rng = np.random.default_rng(5)
    n = 200
    M = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.3)
    A = csr_from_dense(M)
    M32 = M.astype(np.float32).astype(np.float64)
    x32 = rng.standard_normal(n).astype(np.float32)
    ref = M32 @ x32.astype(np.float64)
    L = int(np.diff(A.row_ptr).max())
    gam = L * U32 / (1 - L * U32)
    bound = gam * (np.abs(M32) @ np.abs(x32.astype(np.float64)))
    y = oracle.spmv_f32(A, x32).astype(np.float64)
    assert np.all(np.abs(y - ref) <= bound)
    # float32 rounding really happens: the error is well above float64's bound
    assert np.abs(y - ref).max() > 1e3 * L * EPS * np.abs(ref).max()
    assert np.abs(_spmv_f32_f64_accumulator(A, x32).astype(np.float64) - ref).max() <= \
        U32 * np.abs(ref).max()


def test_dot_small_exact():
    assert oracle.dot(np.array([1.0, 2.0, 3.0]), np.array([4.0, -5.0, 6.0])) == 12.0
    assert oracle.dot(np.zeros(0), np.zeros(0)) == 0.0


def test_row_slice_and_split():
    A = I.poisson2d(10)
    rp, ci, v = oracle.row_slice(A, 13, 57)
    assert rp[0] == 0 and rp[-1] == A.row_ptr[57] - A.row_ptr[13]
    assert np.array_equal(ci, A.col[A.row_ptr[13]:A.row_ptr[57]])
    assert np.array_equal(rp, A.row_ptr[13:58] - A.row_ptr[13])
    assert oracle.split_rows(101, 0.5) == 51      # 50.5 rounds away from zero
    assert oracle.split_rows(100, 0.25) == 25
    assert oracle.split_rows(7, 0.0) == 0 and oracle.split_rows(7, 1.0) == 7


# ----------------------------------------------------------------------------- CG

def test_cg_one_by_one():
    A = I.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    out = oracle.cg(A, np.array([3.0]), tol=1e-14, maxit=5)
    assert out["status"] == oracle.OK and out["iterations"] == 1
    assert out["x"][0] == 0.75


def test_cg_first_step_by_hand():
    M, _ = random_spd_dense(12, 20.0, seed=3)
    A = csr_from_dense(M)
    b = np.random.default_rng(4).standard_normal(12)
    out = oracle.cg(A, b, tol=0.0, maxit=1)
    r0 = b
    x1 = (r0 @ r0) / (r0 @ (M @ r0)) * r0
    np.testing.assert_allclose(out["x"], x1, rtol=1e-13, atol=1e-15)
    assert out["status"] == oracle.MAXIT and out["iterations"] == 1


@pytest.mark.parametrize("n,cond,seed", [(8, 4.0, 0), (16, 10.0, 1), (13, 9.0, 2)])
def test_cg_finite_termination_small_spd(n, cond, seed):
    M, _ = random_spd_dense(n, cond, seed)
    A = csr_from_dense(M)
    b = np.random.default_rng(seed + 10).standard_normal(n)
    out = oracle.cg(A, b, tol=1e-12, maxit=n)
    assert out["status"] == oracle.OK
    assert out["iterations"] <= n
    assert np.linalg.norm(b - M @ out["x"]) <= 1e-12 * np.linalg.norm(b) * 2


def test_cg_k_distinct_eigenvalues_terminates_in_k():
    rng = np.random.default_rng(5)
    n, lam_vals = 40, np.array([1.0, 1.7, 2.5, 4.0, 6.5])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = lam_vals[rng.integers(0, lam_vals.size, n)]
    lam[: lam_vals.size] = lam_vals
    M = (Q * lam) @ Q.T
    A = csr_from_dense(M)
    b = rng.standard_normal(n)
    out = oracle.cg(A, b, tol=1e-10, maxit=n)
    assert out["status"] == oracle.OK and out["iterations"] <= lam_vals.size


def test_cg_identity_plus_low_rank():
    rng = np.random.default_rng(6)
    n, rank = 30, 3
    U = rng.standard_normal((n, rank))
    M = np.eye(n) + U @ U.T
    out = oracle.cg(csr_from_dense(M), rng.standard_normal(n), tol=1e-10, maxit=n)
    assert out["status"] == oracle.OK and out["iterations"] <= rank + 1


def test_cg_matches_dense_solve_and_manufactured_solution():
    p = I.poisson2d_problem(8)
    M = p.A.scipy().toarray()
    out = oracle.cg(p.A, p.b, tol=1e-12, maxit=500)
    assert out["status"] == oracle.OK
    lam = np.linalg.eigvalsh(M)
    kappa = lam[-1] / lam[0]
    err = np.linalg.norm(out["x"] - p.xstar) / np.linalg.norm(p.xstar)
    assert err <= kappa * 1e-12 * 2
    np.testing.assert_allclose(out["x"], np.linalg.solve(M, p.b), rtol=0, atol=kappa * 1e-12)
    true = np.linalg.norm(p.b - M @ out["x"]) / np.linalg.norm(p.b)
    assert abs(true - out["rel_res_true"]) <= 1e-15 + 1e-3 * true


def _poisson2d_kappa(N):
    j = np.arange(1, N + 1)
    lam1 = 2 - 2 * np.cos(j * np.pi / (N + 1))
    return (2 * lam1.max()) / (2 * lam1.min())


def test_cg_a_norm_error_monotone_and_chebyshev_bound():
    N = 16
    p = I.poisson2d_problem(N, seed=9)
    M = p.A.scipy().toarray()
    np.testing.assert_allclose(np.linalg.eigvalsh(M)[[0, -1]],
                               np.sort(np.linalg.eigvalsh(M))[[0, -1]])
    kappa = _poisson2d_kappa(N)
    lam = np.linalg.eigvalsh(M)
    assert abs(lam[-1] / lam[0] - kappa) <= 1e-8 * kappa   # closed-form eigenvalues
    q = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)

    def anorm(e):
        return math.sqrt(e @ (M @ e))

    e0 = anorm(p.xstar)
    prev = e0
    for k in range(1, 60):
        xk = oracle.cg(p.A, p.b, tol=0.0, maxit=k)["x"]
        ek = anorm(xk - p.xstar)
        assert ek <= prev * (1 + 1e-12) + 1e-14 * e0
        assert ek <= 2 * q ** k * e0 * (1 + 1e-9) + 1e-13 * e0
        prev = ek


def test_cg_rho_history_is_residual_norm():
    p = I.poisson2d_problem(12)
    out = oracle.cg(p.A, p.b, tol=1e-10, maxit=400, history=True)
    M = p.A.scipy().toarray()
    for k in (0, 5, 20):
        xk = oracle.cg(p.A, p.b, tol=0.0, maxit=k)["x"]
        rk = p.b - M @ xk
        assert abs(out["rho"][k] - rk @ rk) <= 1e-10 * (p.b @ p.b)
    assert len(out["rho"]) == out["iterations"] + 1


def test_cg_edge_cases():
    p = I.poisson2d_problem(6)
    # b = 0: solution is zero, nothing to iterate
    out = oracle.cg(p.A, np.zeros(p.A.n), x0=np.ones(p.A.n))
    assert out["status"] == oracle.OK and out["iterations"] == 0 and not out["x"].any()
    # maxit = 0: x untouched
    x0 = np.linspace(-1, 1, p.A.n)
    out = oracle.cg(p.A, p.b, x0=x0, maxit=0)
    assert out["status"] == oracle.MAXIT and np.array_equal(out["x"], x0)
    # exact initial guess: converged before any iteration
    out = oracle.cg(I.poisson2d(6), oracle.spmv(I.poisson2d(6), np.ones(36)), x0=np.ones(36))
    assert out["status"] == oracle.OK and out["iterations"] == 0
    # indefinite matrix: breakdown
    B = I.poisson2d(6)
    B.val = B.val.copy()
    B.val[B.col == np.repeat(np.arange(36), np.diff(B.row_ptr))] = -4.0
    out = oracle.cg(B, np.ones(36), maxit=50)
    assert out["status"] == oracle.EBREAKDOWN
    # NaN in b: breakdown
    b = p.b.copy(); b[3] = np.nan
    assert oracle.cg(p.A, b, maxit=10)["status"] == oracle.EBREAKDOWN
    # fixed-work mode (tol = 0) runs exactly maxit iterations
    out = oracle.cg(p.A, p.b, tol=0.0, maxit=7)
    assert out["iterations"] == 7 and out["status"] == oracle.MAXIT


# ----------------------------------------------------------------------------- PCG

def _identity(n):
    return I.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))


def test_pcg_identity_is_plain_cg_bitwise():
    p = I.diffusion_problem(16, seed=3)
    E = _identity(p.A.n)
    a = oracle.cg(p.A, p.b, tol=1e-10, maxit=2000)
    b = oracle.pcg(p.A, E, E, p.b, tol=1e-10, maxit=2000)
    assert a["iterations"] == b["iterations"] and np.array_equal(a["x"], b["x"])


def test_pcg_exact_inverse_factor_converges_in_one_step():
    M, _ = random_spd_dense(20, 1e4, seed=8)
    L = np.linalg.cholesky(M)
    Gd = np.linalg.inv(L)                 # G^T G = L^-T L^-1 = M^-1
    G = csr_from_dense(np.tril(Gd))
    Gt = csr_from_dense(np.tril(Gd).T.copy())
    b = np.random.default_rng(9).standard_normal(20)
    out = oracle.pcg(csr_from_dense(M), G, Gt, b, tol=1e-9, maxit=20)
    assert out["status"] == oracle.OK and out["iterations"] == 1


def test_pcg_jacobi_matches_dense_preconditioned_iteration():
    p = I.diffusion_problem(12, seed=4)
    M = p.A.scipy().toarray()
    d = np.diag(M)
    G = I.CSR(p.A.n, np.arange(p.A.n + 1, dtype=np.int32), np.arange(p.A.n, dtype=np.int32),
              1.0 / np.sqrt(d))
    out = oracle.pcg(p.A, G, G, p.b, tol=0.0, maxit=3)
    # three steps of Jacobi-PCG written densely
    x = np.zeros(p.A.n); r = p.b.copy(); z = r / d; pp = z.copy(); rho = r @ z
    for _ in range(3):
        q = M @ pp; a = rho / (pp @ q); x += a * pp; r -= a * q
        z = r / d; rn = r @ z; pp = z + (rn / rho) * pp; rho = rn
    np.testing.assert_allclose(out["x"], x, rtol=1e-10, atol=1e-12 * np.abs(x).max())
    plain = oracle.cg(p.A, p.b, tol=1e-10, maxit=5000)["iterations"]
    jac = oracle.pcg(p.A, G, G, p.b, tol=1e-10, maxit=5000)["iterations"]
    assert jac < plain


# ----------------------------------------------------------------------------- mixed precision

def test_mixed_reaches_fp64_tolerance():
    p = I.random_spd_problem(4000, seed=21)
    out = oracle.cg_mixed(p.A, p.b, tol=1e-10, maxit=5000)
    assert out["status"] == oracle.OK
    r = p.b - p.A.scipy() @ out["x"]
    assert np.linalg.norm(r) / np.linalg.norm(p.b) < 1e-10
    assert out["fp64_residuals"] >= 2
    ref = oracle.cg(p.A, p.b, tol=1e-12, maxit=5000)["x"]
    # lambda_min = 0.01 exactly (A 1 = 0.01 1, the rest is a graph Laplacian)
    # lambda_max <= largest absolute row sum (Gershgorin)
    lam_max = np.max(np.add.reduceat(np.abs(p.A.val), p.A.row_ptr[:-1]))
    kappa = lam_max / 0.01
    err = np.linalg.norm(out["x"] - ref) / np.linalg.norm(ref)
    assert err <= kappa * 2e-10


def test_mixed_on_fp32_exact_matrix_tracks_fp64_iteration_count():
    p = I.poisson2d_problem(32, seed=5)
    mixed = oracle.cg_mixed(p.A, p.b, tol=1e-10, maxit=2000)
    plain = oracle.cg(p.A, p.b, tol=1e-10, maxit=2000)
    assert mixed["status"] == oracle.OK
    assert mixed["iterations"] <= 1.5 * plain["iterations"]
    assert np.linalg.norm(p.b - p.A.scipy() @ mixed["x"]) / np.linalg.norm(p.b) < 1e-10


def test_mixed_edge_cases():
    p = I.poisson2d_problem(6)
    out = oracle.cg_mixed(p.A, np.zeros(p.A.n))
    assert out["status"] == oracle.OK and out["iterations"] == 0
    out = oracle.cg_mixed(p.A, p.b, maxit=0)
    assert out["status"] == oracle.MAXIT and out["iterations"] == 0
    assert oracle.cg_mixed(p.A, p.b, delta=1.5)["status"] == oracle.EINVAL
