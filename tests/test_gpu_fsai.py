"""GPU parity of the learned FSAI preconditioner and the preconditioned solve.

Bars:
* features: the bfloat16 features equal the oracle's bit for bit, except where
  a last-bit difference of the float64 logarithm moves a value across a
  bfloat16 rounding boundary (then one bfloat16 ulp; at most 0.1% of entries).
* network outputs: max |o - o_ref| <= 2e-3 max |o_ref| (float32 matrix-core
  accumulation against float64 sums of the same bfloat16 operands).
* loss: relative 1e-4; gradient: relative 2-norm error <= 1e-2 and cosine
  >= 0.999 (float32 atomics in the loss backward, bfloat16 re-rounding of the
  back-propagated signals).
* PCG with a given factor: both converge, iteration counts within max(2, 5%)
  of the oracle's PCG with the same factor, ||x - x_ref|| / ||x_ref|| <=
  2 kappa(A) tol.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.fsai as OF
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def field(nx, ny, seed):
    return I.diffusion2d(I.log_normal_field(nx, ny, [seed, 0]))


def theta_with_biases(seed):
    from paper_2608_09647_amd import fsai
    th = fsai.init_params(seed).astype(np.float64)
    rng = np.random.default_rng([seed, 3])
    for lo, hi in ((768, 832), (4928, 4992), (5312, 5317)):
        th[lo:hi] = rng.uniform(-0.2, 0.2, hi - lo)
    return th.astype(np.float32)


def as_csr(M):
    rp, ci, va = OF.csr_parts(M)
    return I.CSR(M.shape[0], rp, ci, va)


def kappa(A):
    ev = np.linalg.eigvalsh(A.scipy().toarray())
    return float(ev[-1] / ev[0])


# ----------------------------------------------------------------------------- features and network

def test_features_match_oracle(cg):
    systems = [field(20, 24, 3), field(33, 17, 4)]
    with_th = theta_with_biases(0)
    tr = cg.FsaiTrainer(systems, with_th)
    for s, A in enumerate(systems):
        print(f"[features] system {s} n={A.n}", flush=True)
        got = tr.features(s).astype(np.float64)
        ref = OF.bf16(OF.features(A))
        diff = got != ref
        assert diff.mean() <= 1e-3
        if diff.any():
            assert np.all(np.abs(got - ref)[diff] <= np.abs(ref)[diff] * 2.0 ** -7)
    tr.close()


def assert_blockwise_close(got, ref, tag, rtol=1e-4):
    """Every parameter block (W1, b1, W2, b2, W3, b3) element by element:
    |got - ref| <= rtol * max |ref block|.  Both sides round the same operands
    to bfloat16 at the same points; the kernel accumulates in float32 and the
    oracle in float64, so entries differ by float32 accumulation error."""
    k = 0
    for name, shape in OF.SHAPES:
        size = int(np.prod(shape))
        gb, rb = got[k:k + size], ref[k:k + size]
        scale = np.abs(rb).max()
        err = np.abs(gb - rb).max()
        print(f"[{tag}] {name}: max |diff| {err:.3e} of max |g| {scale:.3e}", flush=True)
        assert err <= rtol * scale, (name, err, scale)
        k += size
    assert k == got.size == ref.size


def test_forward_outputs_match_oracle(cg):
    A = field(40, 30, 5)
    th = theta_with_biases(1)
    tr = cg.FsaiTrainer([A], th)
    rows = np.arange(0, A.n, 7, dtype=np.int32)[None, :]
    _, _, out = tr.loss_grad([0], rows, outputs=True)
    ref, _ = OF.mlp_forward(th.astype(np.float64), OF.features(A), round_bf16=True)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"[forward] max rel err {err:.3e}", flush=True)
    assert err <= 2e-3
    tr.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_loss_and_gradient_match_oracle(cg, seed):
    A = field(36, 28, 10 + seed)
    th = theta_with_biases(seed)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(A.n, 200, replace=False)).astype(np.int32)
    tr = cg.FsaiTrainer([A], th)
    loss, grad = tr.loss_grad([0], rows[None, :])
    L, g = OF.network_loss(th.astype(np.float64), A, rows, round_bf16=True)
    rel = np.linalg.norm(grad - g) / np.linalg.norm(g)
    cos = float(grad @ g / (np.linalg.norm(grad) * np.linalg.norm(g)))
    print(f"[grad] loss {loss:.6e} ref {L:.6e} grad rel {rel:.3e} cos {cos:.6f}", flush=True)
    assert abs(loss - L) <= 1e-4 * L
    assert_blockwise_close(grad, g, "grad")
    assert rel <= 1e-2 and cos >= 0.999
    # the unused outputs (E, N) get no gradient
    assert grad[5312 + 2] == 0 and grad[5312 + 4] == 0
    tr.close()


def test_multi_system_loss_is_sample_weighted_mean(cg):
    systems = [field(24, 24, 20), field(30, 20, 21), field(16, 40, 22)]
    th = theta_with_biases(2)
    rng = np.random.default_rng(5)
    rows = np.stack([rng.choice(A.n, 96, replace=False) for A in systems]).astype(np.int32)
    tr = cg.FsaiTrainer(systems, th)
    loss, grad = tr.loss_grad([0, 1, 2], rows)
    # the mean over all sampled rows: one backward pass whose bfloat16
    # rounding sees each row's signal with the factor 1/|S| of the whole sample
    L, g = OF.network_loss_multi(th.astype(np.float64), systems, list(rows), round_bf16=True)
    Ls = [OF.network_loss(th.astype(np.float64), A, r, round_bf16=True)[0] for A, r in zip(systems, rows)]
    rel = np.linalg.norm(grad - g) / np.linalg.norm(g)
    print(f"[multi] loss {loss:.6e} ref {L:.6e} grad rel {rel:.3e}", flush=True)
    assert abs(loss - L) <= 1e-4 * L and rel <= 1e-2
    assert_blockwise_close(grad, g, "multi")
    # a subset of systems in another order gives the same as those systems alone
    loss2, _ = tr.loss_grad([2, 0], rows[[2, 0]])
    assert abs(loss2 - (Ls[2] + Ls[0]) / 2) <= 1e-4 * loss2
    tr.close()


def test_adam_steps_match_oracle(cg):
    A = field(32, 32, 30)
    th = theta_with_biases(3)
    rows = np.arange(0, A.n, 5, dtype=np.int32)[None, :]
    tr = cg.FsaiTrainer([A], th)
    lr = 1e-3
    theta = th.astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in (1, 2):
        _, g = tr.loss_grad([0], rows, theta=theta.astype(np.float32))
        tr.step([0], rows, lr)
        theta, m, v = OF.adam_step(theta, m, v, g.astype(np.float64), t, lr=lr)
        got = tr.params().astype(np.float64)
        print(f"[adam] step {t} max diff {np.abs(got - theta).max():.3e}", flush=True)
        assert np.abs(got - theta).max() <= 2e-2 * lr
        theta = got
    tr.close()


# ----------------------------------------------------------------------------- factor and PCG

def test_learned_factor_matches_oracle(cg):
    A = field(48, 40, 40)
    th = theta_with_biases(4)
    with cg.Solver(A) as s:
        s.fsai_setup(th)
        rp, ci, va = s.read_factor()
    o, _ = OF.mlp_forward(th.astype(np.float64), OF.features(A), round_bf16=True)
    Gt = OF.g_tilde(A, o)
    _, d = OF.scaled_operator(A)
    G = OF.g_unscaled(Gt, d).tocsr()
    G.sort_indices()
    assert np.array_equal(rp, G.indptr) and np.array_equal(ci, G.indices)
    L = sp.tril(A.scipy()).tocsr()
    L.sort_indices()
    assert np.array_equal(rp, L.indptr) and np.array_equal(ci, L.indices)
    err = np.abs(va - G.data).max() / np.abs(G.data).max()
    print(f"[factor] max rel err {err:.3e}", flush=True)
    assert err <= 2e-3


def test_learned_factor_on_an_unsymmetric_pattern(cg):
    """G^T's structure comes from A's upper triangle only where A's pattern
    is symmetric.  With one entry above the diagonal missing (its mirror
    kept), the setup transposes G instead: the factor is still on tril(A),
    and fixed PCG steps equal those with the same factor installed from the
    host (whose G^T is always transposed); with the pattern symmetric again
    the same holds on the direct path."""
    A = field(40, 36, 54)
    M = A.scipy().tolil()
    M[100, 101] = 0.0
    M = M.tocsr()
    M.eliminate_zeros()
    M.sort_indices()
    A2 = I.CSR(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))
    b = I.rhs_of(A, I.uniform_vector(A.n, [54, 1]))
    th = theta_with_biases(6)
    for Am in (A2, A):
        with cg.Solver(Am) as s:
            s.fsai_setup(th)
            rp, ci, va = s.read_factor()
        L = sp.tril(Am.scipy()).tocsr()
        L.sort_indices()
        assert np.array_equal(rp, L.indptr) and np.array_equal(ci, L.indices)
        G = sp.csr_matrix((va, ci, rp), shape=(Am.n, Am.n))
        x1, r1 = run_pcg(cg, Am, b, theta=th, tol=0.0, maxit=40)
        x2, r2 = run_pcg(cg, Am, b, G=as_csr(G), tol=0.0, maxit=40)
        assert r1["iterations"] == r2["iterations"] and r1["fell_back"] == r2["fell_back"]
        assert np.array_equal(x1, x2)


def run_pcg(cg, A, b, G=None, theta=None, tol=1e-10, maxit=20000, x0=None, **opts):
    with cg.Solver(A) as s:
        if G is not None:
            s.set_fsai(G)
        else:
            s.fsai_setup(theta)
        s.set_opts(precond=cg.PC_FSAI, **opts)
        x = dev(np.zeros(A.n) if x0 is None else x0)
        x, res = s.solve(dev(b), x, tol=tol, maxit=maxit)
        return host(x), res


def check_pcg_against_oracle(cg, A, b, G, tol=1e-10):
    Gc = as_csr(G)
    Gtc = as_csr(sp.csr_matrix(G).T.tocsr())
    ref = oracle.pcg(A, Gc, Gtc, b, tol=tol, maxit=20000)
    x, res = run_pcg(cg, A, b, G=Gc, tol=tol)
    print(f"[pcg] gpu it={res['iterations']} status={res['status']} rel={res['rel_res_true']:.2e} "
          f"| oracle it={ref['iterations']} status={ref['status']}", flush=True)
    assert ref["status"] == 0 and res["status"] == 0 and res["converged"] == 1
    assert res["fell_back"] == 0
    assert abs(res["iterations"] - ref["iterations"]) <= max(2, 0.05 * ref["iterations"])
    assert res["rel_res_true"] <= tol * 1.01
    k = kappa(A)
    assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"]) <= 2 * k * tol
    return res, ref


def test_pcg_identity_factor_tracks_plain_cg(cg):
    p = I.poisson2d_problem(40, seed=1)
    E = sp.identity(p.A.n, format="csr")
    res, ref = check_pcg_against_oracle(cg, p.A, p.b, E)
    plain = oracle.cg(p.A, p.b, tol=1e-10, maxit=20000)
    assert ref["iterations"] == plain["iterations"]


def test_pcg_jacobi_factor_matches_oracle(cg):
    A = field(40, 40, 50)
    b = I.rhs_of(A, I.uniform_vector(A.n, [50, 1]))
    d = A.scipy().diagonal()
    check_pcg_against_oracle(cg, A, b, sp.diags(1.0 / np.sqrt(d)).tocsr())


def test_pcg_classic_fsai_matches_oracle(cg):
    A = field(40, 36, 51)
    b = I.rhs_of(A, I.uniform_vector(A.n, [51, 1]))
    res, ref = check_pcg_against_oracle(cg, A, b, OF.classic_fsai(A))
    plain = oracle.cg(A, b, tol=1e-10, maxit=20000)
    assert ref["iterations"] < plain["iterations"]


def random_lower_factor(n, per_row, seed):
    """Lower-triangular factor with up to `per_row` entries per row at random
    columns (positive diagonal, so M = G^T G is SPD): 64-row slices use far
    more than 8 column offsets, so it stays in CSR."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        k = min(i, per_row - 1)
        cs = list(rng.choice(i, size=k, replace=False)) if k > 0 else []
        rows += [i] * (k + 1)
        cols += cs + [i]
        vals += list(rng.uniform(-0.2, 0.2, k)) + [1.0 + rng.random()]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("per_row", [4, 12])
def test_pcg_scattered_factor_matches_oracle(cg, per_row):
    """A factor that does not fit stencil slices: the CSR form of the fused
    r/t kernel (at most 8 entries per row), or the unfused x/r update, SpMV
    with G and p update (more)."""
    p = I.poisson2d_problem(40, seed=2)
    check_pcg_against_oracle(cg, p.A, p.b, random_lower_factor(p.A.n, per_row, 11))


def test_pcg_learned_factor_matches_oracle_with_same_factor(cg):
    A = field(44, 44, 52)
    b = I.rhs_of(A, I.uniform_vector(A.n, [52, 1]))
    th = theta_with_biases(5)
    with cg.Solver(A) as s:
        s.fsai_setup(th)
        rp, ci, va = s.read_factor()
    G = sp.csr_matrix((va, ci, rp), shape=(A.n, A.n))
    check_pcg_against_oracle(cg, A, b, G)
    # the learned path itself (factor built on the device) gives the same run
    x, res = run_pcg(cg, A, b, theta=th)
    x2, res2 = run_pcg(cg, A, b, G=as_csr(G))
    assert res["iterations"] == res2["iterations"] and np.array_equal(x, x2)


@pytest.mark.parametrize("maxit,tol", [(1, 0.0), (2, 0.0), (7, 0.0), (20000, 1e-10)])
def test_pcg_fused_direction_update_is_bitwise(cg, maxit, tol):
    """cg_opts.fuse_dir with the learned factor: the end of iteration k
    (r^T z, beta, the stop test, x += alpha p_k, p_{k+1} = z + beta p_k)
    inside the SpMV of iteration k+1 gives bitwise the separate kernels' x,
    iterations and residuals (odd row count; stops at odd and even
    iterations), and SpMV event sampling counts the same launches."""
    A = field(61, 47, 53)
    b = I.rhs_of(A, I.uniform_vector(A.n, [53, 1]))
    th = theta_with_biases(5)
    x0, r0 = run_pcg(cg, A, b, theta=th, tol=tol, maxit=maxit, fuse_dir=cg.FUSE_OFF, profile=3)
    x1, r1 = run_pcg(cg, A, b, theta=th, tol=tol, maxit=maxit, fuse_dir=cg.FUSE_ON, profile=3)
    assert r0["fused_dir"] == 0 and r1["fused_dir"] == 1 and r1["spmv_kind"] == 6
    assert r0["status"] == r1["status"] and r0["iterations"] == r1["iterations"]
    assert r0["rel_res_recur"] == r1["rel_res_recur"] and r0["rel_res_true"] == r1["rel_res_true"]
    assert np.array_equal(x0, x1)
    assert r0["n_spmv"] == r1["n_spmv"] == (min(maxit, r1["iterations"]) + 2) // 3


def test_pcg_breakdown_falls_back_to_plain_cg(cg):
    p = I.poisson2d_problem(24, seed=1)
    G = sp.identity(p.A.n, format="lil")
    G[3, 3] = np.nan
    x, res = run_pcg(cg, p.A, p.b, G=as_csr(G.tocsr()))
    plain = oracle.cg(p.A, p.b, tol=1e-10, maxit=20000)
    assert res["fell_back"] == 1 and res["status"] == 0 and res["converged"] == 1
    assert abs(res["iterations"] - plain["iterations"]) <= max(2, 0.05 * plain["iterations"])
    assert np.all(np.isfinite(x))


def test_pcg_edge_cases(cg):
    p = I.poisson2d_problem(20, seed=1)
    E = as_csr(sp.identity(p.A.n, format="csr"))
    # b = 0 -> x = 0
    x, res = run_pcg(cg, p.A, np.zeros(p.A.n), G=E, x0=np.ones(p.A.n))
    assert res["status"] == 0 and not x.any()
    # x0 = solution -> no iteration
    x, res = run_pcg(cg, p.A, p.b, G=E, x0=p.xstar, tol=1e-8)
    assert res["iterations"] == 0 and res["status"] == 0
    # maxit = 0 -> not converged, x unchanged
    x, res = run_pcg(cg, p.A, p.b, G=E, maxit=0)
    assert res["status"] == cg.CG_MAXIT and res["iterations"] == 0 and not x.any()
    # fixed work (tol = 0) runs exactly maxit iterations
    x, res = run_pcg(cg, p.A, p.b, G=E, tol=0.0, maxit=37, check_every=8)
    ref = oracle.pcg(p.A, E, E, p.b, tol=0.0, maxit=37)
    assert res["iterations"] == 37 and ref["iterations"] == 37
    assert np.linalg.norm(x - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])


def test_fsai_rejects_non_stencil_and_split_handles(cg):
    A = I.random_spd_lognormal(2000, seed=3)
    with cg.Solver(A) as s:
        with pytest.raises(cg.CgError):
            s.fsai_setup(theta_with_biases(0))
        with pytest.raises(cg.CgError):
            s.set_opts(precond=cg.PC_FSAI)
            s.solve(dev(np.ones(A.n)))
    p = I.poisson2d_problem(16, seed=1)
    with cg.Solver(p.A, 0, p.A.n // 2) as s:
        with pytest.raises(cg.CgError):
            s.set_fsai(sp.identity(p.A.n, format="csr"))
        with pytest.raises(cg.CgError):
            s.set_opts(precond=cg.PC_FSAI)


# ----------------------------------------------------------------------------- training gain

def test_training_reduces_loss_and_beats_plain_cg(cg):
    from paper_2608_09647_amd import fsai
    systems = fsai.training_systems(48, nx=32, first=0)
    tr = cg.FsaiTrainer(systems, fsai.init_params(0))
    hist = fsai.train(tr, steps=400, nsel=8, rows_per=256, lr=3e-3, lr_final=3e-4, seed=0)
    L = hist["losses"]
    print(f"[train] loss {np.mean(L[:10]):.4e} -> {np.mean(L[-10:]):.4e} in {hist['seconds']:.2f}s",
          flush=True)
    assert np.mean(L[-10:]) < 0.5 * np.mean(L[:10])
    theta = tr.params()
    tr.close()
    p = I.diffusion_problem(64, seed=10_000)
    plain = oracle.cg(p.A, p.b, tol=1e-10, maxit=50000)
    x, res = run_pcg(cg, p.A, p.b, theta=theta)
    # the same network before training: what training itself gains
    _, res0 = run_pcg(cg, p.A, p.b, theta=fsai.init_params(0))
    print(f"[gain] plain {plain['iterations']} untrained {res0['iterations']} learned {res['iterations']}",
          flush=True)
    assert res["status"] == 0 and res["fell_back"] == 0
    assert res["iterations"] < plain["iterations"]
    assert res["iterations"] < res0["iterations"]
    assert res["rel_res_true"] <= 1.01e-10


def test_training_is_reproducible(cg):
    """dL/dG~ is summed in fixed point, so the order in which the loss
    kernel's atomics land does not change it: two trainers with the same
    initial parameters and samples end bit for bit alike (losses included),
    and the fixed-point gradient stays within the float bar of the oracle's
    (the loss/gradient parity tests above)."""
    from paper_2608_09647_amd import fsai
    systems = fsai.training_systems(12, nx=32, first=0)
    runs = []
    for _ in range(2):
        tr = cg.FsaiTrainer(systems, fsai.init_params(0))
        hist = fsai.train(tr, steps=60, nsel=4, rows_per=256, lr=3e-3, seed=1)
        runs.append((tr.params(), np.asarray(hist["losses"])))
        tr.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


# ----------------------------------------------------------------------------- classic FSAI

CLASSIC_CASES = {
    "diffusion_40x36": lambda: field(40, 36, 51),
    "poisson3d_12": lambda: I.poisson3d(12),
    # tril rows of 8 entries at most (the classic factor's limit)
    "random_short_rows": lambda: I.random_spd_lognormal(1500, 2, mean_degree=1.5, sigma=0.2, max_degree=2,
                                                        shift=1.0),
}


@pytest.mark.parametrize("name", list(CLASSIC_CASES))
def test_classic_fsai_factor_matches_oracle(cg, name):
    A = CLASSIC_CASES[name]()
    ref = OF.classic_fsai(A)
    with cg.Solver(A) as s:
        s.fsai_classic()
        rp, ci, va = s.read_factor()
    assert np.array_equal(rp, ref.indptr) and np.array_equal(ci, ref.indices)
    # per-row local solves: Cholesky here, LU in the oracle
    scale = np.repeat(np.maximum.reduceat(np.abs(ref.data), ref.indptr[:-1]), np.diff(ref.indptr))
    err = np.max(np.abs(va - ref.data) / scale)
    print(f"[classic] {name}: max row-relative difference {err:.2e}", flush=True)
    assert err <= 1e-12
    # unit diagonal of G A G^T (the defining property of the scaling)
    G = sp.csr_matrix((va, ci, rp), shape=(A.n, A.n))
    d = (G @ A.scipy() @ G.T).diagonal()
    assert np.max(np.abs(d - 1.0)) <= 1e-12


def test_pcg_with_classic_factor_matches_oracle(cg):
    A = field(40, 40, 53)
    b = I.rhs_of(A, I.uniform_vector(A.n, [53, 1]))
    with cg.Solver(A) as s:
        s.fsai_classic()
        s.set_opts(precond=cg.PC_FSAI)
        x, res = s.solve(dev(b), tol=1e-10, maxit=20000)
        rp, ci, va = s.read_factor()
    res2, ref = check_pcg_against_oracle(cg, A, b, sp.csr_matrix((va, ci, rp), shape=(A.n, A.n)))
    assert res["iterations"] == res2["iterations"]
    plain = oracle.cg(A, b, tol=1e-10, maxit=20000)
    assert ref["iterations"] < plain["iterations"]


def test_classic_fsai_rejections(cg):
    long_rows = I.random_spd_lognormal(500, 0)                 # tril rows far longer than 8
    with cg.Solver(long_rows) as s:
        with pytest.raises(cg.CgError, match="more than"):
            s.fsai_classic()
    no_diag = I.poisson2d(6)
    keep = no_diag.col != np.repeat(np.arange(no_diag.n), np.diff(no_diag.row_ptr))
    keep[np.flatnonzero(~keep)[1:]] = True                     # drop the diagonal of row 0 only
    rows = np.repeat(np.arange(no_diag.n), np.diff(no_diag.row_ptr))[keep]
    M = I.CSR(no_diag.n, np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=no_diag.n))]).astype(np.int32),
              no_diag.col[keep], no_diag.val[keep])
    with cg.Solver(M) as s:
        with pytest.raises(cg.CgError, match="no diagonal"):
            s.fsai_classic()
    neg = I.poisson2d(6)
    neg.val = np.where(neg.col == np.repeat(np.arange(neg.n), np.diff(neg.row_ptr)), -4.0, neg.val)
    with cg.Solver(neg) as s:
        with pytest.raises(cg.CgError, match="not positive definite"):
            s.fsai_classic()


def test_checkpoint_round_trip_and_resume(cg, tmp_path):
    """A checkpoint (theta, Adam m and v, step, seed in an .npz) restores the
    optimiser state bit for bit into a fresh trainer; training 3 steps,
    checkpointing, restoring and training 3 more follows the run of 6 steps
    straight bit for bit (same samples and learning rates; the loss gradient
    is summed in fixed point, independent of the order of its atomics)."""
    from paper_2608_09647_amd import fsai
    systems = [field(32, 32, 50 + k) for k in range(4)]
    th = fsai.init_params(4)
    kw = dict(nsel=2, rows_per=128, lr=1e-3, lr_final=5e-4, seed=9)
    tr = cg.FsaiTrainer(systems, th)
    full = fsai.train(tr, 6, **kw)
    ref = tr.state()
    tr.close()
    tr = cg.FsaiTrainer(systems, th)
    first = fsai.train(tr, 3, total=6, **kw)
    saved = tr.state()
    path = str(tmp_path / "fsai.npz")
    fsai.save_checkpoint(path, tr, seed=kw["seed"], lr=kw["lr"])
    tr.close()
    tr = cg.FsaiTrainer(systems, fsai.init_params(123))   # another start: the checkpoint replaces it
    ck = fsai.load_checkpoint(path, tr)
    assert ck["step"] == 3 and ck["seed"] == 9 and float(ck["lr"]) == kw["lr"]
    back = tr.state()
    assert back["step"] == 3
    for k in ("theta", "m", "v"):
        assert np.array_equal(back[k], saved[k]), k
    rest = fsai.train(tr, 3, start=ck["step"], total=6, **kw)
    got = tr.state()
    tr.close()
    assert got["step"] == ref["step"] == 6
    assert first["losses"] + rest["losses"] == full["losses"]
    for k in ("theta", "m", "v"):
        assert np.array_equal(got[k], ref[k]), k
