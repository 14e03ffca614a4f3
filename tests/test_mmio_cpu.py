"""Matrix Market reader of the library (host code, no GPU): hand-made files
with known CSR, scipy's reader on seeded random files, and every rejected
input."""
import os

import numpy as np
import pytest
import scipy.io
import scipy.sparse as sp


@pytest.fixture(scope="module")
def cg():
    from paper_2608_09647_amd import cgmi
    if not os.path.exists(cgmi.LIB_PATH):
        pytest.skip("libcgmi.so not built")
    return cgmi


def write(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_general_file_sums_repeats_and_sorts_columns(cg, tmp_path):
    path = write(tmp_path, "g.mtx", """%%MatrixMarket matrix coordinate real general
% a comment
%
3 3 5
3 1 2.5
1 3 -1
1 1 4
2 2 3e0
1 1 0.5
""")
    A, info = cg.read_matrix_market(path)
    assert A.n == 3 and info == {"symmetric": False, "file_entries": 5}
    assert A.row_ptr.tolist() == [0, 2, 3, 4]
    assert A.col.tolist() == [0, 2, 1, 0]
    assert A.val.tolist() == [4.5, -1.0, 3.0, 2.5]


def test_symmetric_file_is_expanded(cg, tmp_path):
    path = write(tmp_path, "s.mtx", """%%MatrixMarket matrix coordinate real symmetric
4 4 6
1 1 4
2 1 -1
2 2 4
3 2 -1
3 3 4
4 4 2
""")
    A, info = cg.read_matrix_market(path)
    dense = np.array([[4, -1, 0, 0], [-1, 4, -1, 0], [0, -1, 4, 0], [0, 0, 0, 2]], float)
    assert info["symmetric"] and info["file_entries"] == 6 and A.nnz == 8
    assert np.array_equal(A.scipy().toarray(), dense)
    for i in range(A.n):
        assert np.all(np.diff(A.col[A.row_ptr[i]:A.row_ptr[i + 1]]) > 0)


def test_pattern_and_integer_fields(cg, tmp_path):
    A, _ = cg.read_matrix_market(write(tmp_path, "p.mtx", """%%MatrixMarket matrix coordinate pattern general
2 2 3
1 1
2 1
2 2
"""))
    assert A.row_ptr.tolist() == [0, 1, 3] and A.col.tolist() == [0, 0, 1] and A.val.tolist() == [1, 1, 1]
    A, _ = cg.read_matrix_market(write(tmp_path, "i.mtx", """%%MATRIXMARKET Matrix Coordinate Integer Symmetric
2 2 2
1 1 7
2 1 -3
"""))
    assert np.array_equal(A.scipy().toarray(), [[7, -3], [-3, 0]])


def test_repeats_are_summed_in_file_order(cg, tmp_path):
    # (1e16 + 1) - 1e16 is 0 in float64; another order would give 1
    path = write(tmp_path, "o.mtx", """%%MatrixMarket matrix coordinate real general
1 1 3
1 1 1e16
1 1 1
1 1 -1e16
""")
    A, _ = cg.read_matrix_market(path)
    assert A.nnz == 1 and A.val[0] == (1e16 + 1.0) - 1e16 == 0.0


def test_empty_rows_and_crlf_line_ends(cg, tmp_path):
    path = str(tmp_path / "c.mtx")
    with open(path, "wb") as f:
        f.write(b"%%MatrixMarket matrix coordinate real general\r\n5 5 2\r\n5 5 1.5\r\n\r\n1 2 2\r\n")
    A, _ = cg.read_matrix_market(path)
    assert A.row_ptr.tolist() == [0, 1, 1, 1, 1, 2] and A.col.tolist() == [1, 4]


@pytest.mark.parametrize("symmetry", ["general", "symmetric"])
def test_matches_scipy_on_random_files(cg, tmp_path, symmetry):
    rng = np.random.default_rng(11)
    n = 3000
    M = sp.random(n, n, density=0.002, random_state=rng, format="coo")
    M.data = rng.standard_normal(M.nnz) * 10.0 ** rng.integers(-8, 8, M.nnz)
    if symmetry == "symmetric":
        M = sp.tril(M + M.T, format="coo")
    path = str(tmp_path / f"r_{symmetry}.mtx")
    scipy.io.mmwrite(path, M, symmetry=symmetry, precision=17)
    A, info = cg.read_matrix_market(path)
    ref = scipy.io.mmread(path).tocsr()
    ref.sum_duplicates()
    ref.sort_indices()
    assert info["symmetric"] == (symmetry == "symmetric")
    assert np.array_equal(A.row_ptr, ref.indptr) and np.array_equal(A.col, ref.indices)
    assert np.array_equal(A.val, ref.data)


def test_thread_count_does_not_change_the_result(cg, tmp_path):
    rng = np.random.default_rng(5)
    n, L = 20000, 200000
    rows, cols = rng.integers(1, n + 1, L), rng.integers(1, n + 1, L)
    vals = rng.standard_normal(L)
    path = str(tmp_path / "big.mtx")
    with open(path, "w") as f:
        f.write(f"%%MatrixMarket matrix coordinate real general\n{n} {n} {L}\n")
        f.writelines(f"{i} {j} {float(v)!r}\n" for i, j, v in zip(rows, cols, vals))
    outs = [cg.read_matrix_market(path, threads=t)[0] for t in (1, 3, 8)]
    for A in outs[1:]:
        assert np.array_equal(A.row_ptr, outs[0].row_ptr) and np.array_equal(A.col, outs[0].col)
        assert np.array_equal(A.val, outs[0].val)
    ref = sp.coo_matrix((vals, (rows - 1, cols - 1)), shape=(n, n)).tocsr()
    ref.sum_duplicates()
    assert np.array_equal(outs[0].row_ptr, ref.indptr) and np.array_equal(outs[0].col, ref.indices)
    assert np.allclose(outs[0].val, ref.data, rtol=1e-15, atol=0)


BAD = {
    "array": "%%MatrixMarket matrix array real general\n2 2\n1\n2\n3\n4\n",
    "complex": "%%MatrixMarket matrix coordinate complex general\n1 1 1\n1 1 1 0\n",
    "skew": "%%MatrixMarket matrix coordinate real skew-symmetric\n2 2 1\n2 1 1\n",
    "hermitian": "%%MatrixMarket matrix coordinate real hermitian\n2 2 1\n2 1 1\n",
    "not_square": "%%MatrixMarket matrix coordinate real general\n2 3 1\n1 1 1\n",
    "no_header": "2 2 1\n1 1 1\n",
    "index_high": "%%MatrixMarket matrix coordinate real general\n2 2 1\n3 1 1\n",
    "index_zero": "%%MatrixMarket matrix coordinate real general\n2 2 1\n0 1 1\n",
    "too_few": "%%MatrixMarket matrix coordinate real general\n2 2 3\n1 1 1\n2 2 1\n",
    "too_many": "%%MatrixMarket matrix coordinate real general\n2 2 1\n1 1 1\n2 2 1\n",
    "no_value": "%%MatrixMarket matrix coordinate real general\n2 2 1\n1 1\n",
    "junk": "%%MatrixMarket matrix coordinate real general\n2 2 1\n1 1 1 x\n",
    "bad_size": "%%MatrixMarket matrix coordinate real general\n2 2\n1 1 1\n",
    "no_size": "%%MatrixMarket matrix coordinate real general\n% only comments\n",
}


@pytest.mark.parametrize("case", sorted(BAD))
def test_rejected_inputs(cg, tmp_path, case):
    path = write(tmp_path, f"{case}.mtx", BAD[case])
    with pytest.raises(cg.CgError) as e:
        cg.read_matrix_market(path)
    assert e.value.code == cg.CG_EINVAL


def test_missing_and_empty_files(cg, tmp_path):
    with pytest.raises(cg.CgError):
        cg.read_matrix_market(str(tmp_path / "absent.mtx"))
    with pytest.raises(cg.CgError):
        cg.read_matrix_market(write(tmp_path, "empty.mtx", ""))
