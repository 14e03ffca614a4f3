"""cg_solve_noalloc (the entry point whose work memory is the library's
static scratch) against cg_solve on the same handle: two calls in a row, the
second on a smaller system, each bit for bit equal to cg_solve; then the
single-workgroup size, fixed work, and the size limit."""
import numpy as np
import pytest

from paper_2608_09647_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cg(require_gpu):
    from paper_2608_09647_amd import cgmi
    cgmi.lib()
    return cgmi


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def both(cg, p, tol, maxit, **opts):
    """(x, result) of cg_solve and of cg_solve_noalloc on one handle."""
    b = dev(p.b)
    with cg.Solver(p.A) as s:
        if opts:
            s.set_opts(**opts)
        x_ref, r_ref = s.solve(b, torch.zeros_like(b), tol=tol, maxit=maxit)
        x_na, r_na = s.solve_noalloc(b, torch.zeros_like(b), tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    return x_ref, r_ref, x_na, r_na


def same(r_ref, r_na, x_ref, x_na):
    assert r_na["code"] == r_ref["code"]
    assert r_na["iterations"] == r_ref["iterations"]
    assert r_na["rel_res_recur"] == r_ref["rel_res_recur"]
    assert r_na["rel_res_true"] == r_ref["rel_res_true"]
    assert r_na["spmv_kind"] == r_ref["spmv_kind"]
    assert torch.equal(x_na, x_ref)


def test_noalloc_matches_cg_solve_twice_second_smaller(cg):
    big = I.poisson2d_problem(1100, seed=1)            # n = 1,210,000: most of the scratch
    small = I.random_spd_problem(30_000, seed=5)
    for name, p in (("poisson2d_1100", big), ("random_spd_30k", small)):
        print(f"[noalloc] {name} n={p.A.n}", flush=True)
        x_ref, r_ref, x_na, r_na = both(cg, p, 1e-10, 100_000 if name == "random_spd_30k" else 60)
        same(r_ref, r_na, x_ref, x_na)
        print(f"[noalloc] {name}: {r_na['iterations']} iterations, code {r_na['code']}, "
              f"true rel. res {r_na['rel_res_true']:.3e}", flush=True)
    assert r_na["code"] == cg.CG_OK


def test_noalloc_single_workgroup_and_fixed_work(cg):
    p = I.poisson2d_problem(48, seed=1)                # n = 2,304: one-workgroup path
    x_ref, r_ref, x_na, r_na = both(cg, p, 1e-10, 5000)
    same(r_ref, r_na, x_ref, x_na)
    assert r_na["code"] == cg.CG_OK
    q = I.poisson3d_problem(40)                        # fixed work, odd iteration count
    x_ref, r_ref, x_na, r_na = both(cg, q, 0.0, 37)
    same(r_ref, r_na, x_ref, x_na)
    assert r_na["iterations"] == 37 and r_na["code"] == cg.CG_MAXIT


def test_noalloc_rejects_what_it_cannot_hold(cg):
    n = 1_700_000                                      # above the scratch's row limit
    A = I.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with cg.Solver(A) as s:
        _, res = s.solve_noalloc(b, x, check=False)
        assert res["code"] == cg.CG_EINVAL and "at most" in cg.last_error()
        # the handle still works through cg_solve
        _, res = s.solve(b, x, tol=1e-10)
        assert res["code"] == cg.CG_OK
    p = I.poisson2d_problem(40)
    with cg.Solver(p.A) as s:
        s.set_opts(precision=cg.PREC_MIXED)
        _, res = s.solve_noalloc(dev(p.b), torch.zeros(p.A.n, dtype=torch.float64, device="cuda"),
                                 check=False)
        assert res["code"] == cg.CG_EINVAL
    with cg.Solver(p.A, 0, 800) as s:                  # a split handle
        _, res = s.solve_noalloc(dev(p.b), torch.zeros(p.A.n, dtype=torch.float64, device="cuda"),
                                 check=False)
        assert res["code"] == cg.CG_EINVAL
