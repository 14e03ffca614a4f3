"""Properties of the seeded synthetic inputs (closed forms, symmetry, determinism)."""
import numpy as np
import pytest

from paper_2608_09647_amd import inputs as I


def _check_csr(A):
    rp = A.row_ptr.astype(np.int64)
    assert A.row_ptr.dtype == np.int32 and A.col.dtype == np.int32 and A.val.dtype == np.float64
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == A.col.size == A.val.size
    assert A.col.min() >= 0 and A.col.max() < A.n
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    same_row = rows[1:] == rows[:-1]
    assert np.all(A.col[1:][same_row] > A.col[:-1][same_row])   # sorted, unique


def _symmetric_bitwise(A):
    S = A.scipy()
    T = S.T.tocsr()
    T.sort_indices()
    return np.array_equal(S.indptr, T.indptr) and np.array_equal(S.indices, T.indices) \
        and np.array_equal(S.data, T.data)


def test_poisson_closed_forms():
    A = I.poisson2d(64)
    assert (A.n, A.nnz) == (4096, 20224)
    _check_csr(A)
    assert _symmetric_bitwise(A)
    B = I.poisson3d(24)
    assert B.nnz == 7 * B.n - 6 * 24 * 24
    _check_csr(B)
    assert _symmetric_bitwise(B)
    # the full-size 3D closed form: 7 n - 6 * 256^2
    assert 7 * 256 ** 3 - 6 * 256 ** 2 == 117_047_296


def test_diffusion_closed_forms_and_symmetry():
    k = I.log_normal_field(40, 40, [3, 0])
    A = I.diffusion2d(k)
    assert A.nnz == 5 * A.n - 4 * 40
    _check_csr(A)
    assert _symmetric_bitwise(A)
    # row sums = boundary transmissibilities (2 k on each outside face)
    S = A.scipy()
    rs = S @ np.ones(A.n)
    kk = k.reshape(-1)
    ix, iy = np.arange(A.n) % 40, np.arange(A.n) // 40
    bnd = 2 * kk * ((ix == 0).astype(int) + (ix == 39) + (iy == 0) + (iy == 39))
    np.testing.assert_allclose(rs, bnd, rtol=1e-12, atol=1e-12 * np.abs(A.val).max())


def test_field_marginals_are_lognormal():
    k = I.log_normal_field(256, 256, [1, 0])
    z = np.log(k) / 2.0
    assert abs(z.mean()) < 0.2 and abs(z.std() - 1.0) < 0.2
    w = I.gaussian_weights(4.0, 16)
    assert abs(np.sum(w * w) - 1.0) < 1e-14 and w.size == 33


def test_random_spd_properties():
    A = I.random_spd_lognormal(20000, seed=3)
    _check_csr(A)
    assert _symmetric_bitwise(A)
    S = A.scipy()
    np.testing.assert_allclose(S @ np.ones(A.n), 0.01, atol=1e-11)
    d = S.diagonal()
    off = np.add.reduceat(np.abs(A.val), A.row_ptr[:-1]) - d
    np.testing.assert_allclose(d, off + 0.01, rtol=1e-14)
    assert 50 < A.nnz / A.n < 72      # ~30 drawn + ~30 mirrored + diagonal


def test_determinism():
    a = I.random_spd_lognormal(3000, seed=5)
    b = I.random_spd_lognormal(3000, seed=5)
    c = I.random_spd_lognormal(3000, seed=6)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert not (a.nnz == c.nnz and np.array_equal(a.col, c.col))
    p1, p2 = I.poisson2d_problem(16, seed=1), I.poisson2d_problem(16, seed=1)
    assert np.array_equal(p1.b, p2.b) and np.array_equal(p1.xstar, p2.xstar)
    assert p1.xstar.min() >= -1 and p1.xstar.max() <= 1


def test_batch_sides_and_shapes():
    sides = I.batch_sides(256, seed=5)
    assert sides.min() >= 32 and sides.max() <= 512 and sides.size == 256
    probs = I.batch_problem(nsys=3, nrhs=4, sides=[8, 5, 11])
    assert [p.A.n for p in probs] == [64, 25, 121]
    assert probs[1].b.shape == (25, 4)
    np.testing.assert_allclose(probs[2].b, probs[2].A.scipy() @ probs[2].xstar)
