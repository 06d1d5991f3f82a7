"""Matrix Market loader (the paper's matrices come from the SuiteSparse collection in
this format; Section 3, Table 1).  Hand-written fixtures under tests/golden/mtx with
their expected CSR written out here; scipy's reader as a second opinion; the result
passes the library's CSR structure check; malformed files are rejected."""
import os

import numpy as np
import pytest
import scipy.io
import scipy.sparse as sp

import paper_2404_13216_amd as pk
from paper_2404_13216_amd import mtx

GOLD = os.path.join(os.path.dirname(__file__), "golden", "mtx")

EXPECT = {
    "general_dup.mtx": (4, [0, 2, 4, 6, 7], [0, 3, 1, 2, 0, 2, 3], [4.0, -1.25, 5.0, 1.75, -2.0, 0.0, 2.0]),
    "symmetric.mtx": (3, [0, 2, 5, 7], [0, 1, 0, 1, 2, 1, 2], [2.0, -1.0, -1.0, 2.0, -1.0, -1.0, 2.0]),
    "pattern.mtx": (3, [0, 1, 2, 4], [0, 1, 0, 2], [1.0, 1.0, 1.0, 1.0]),
    "integer_skew.mtx": (3, [0, 1, 3, 4], [1, 0, 2, 1], [-3.0, 3.0, 7.0, -7.0]),
}


@pytest.mark.parametrize("name", sorted(EXPECT))
def test_fixture_csr(name):
    A = mtx.read_matrix_market(os.path.join(GOLD, name))
    n, rp, ci, va = EXPECT[name]
    assert A.n == n
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32 and A.val.dtype == np.float64
    assert A.row_ptr.tolist() == rp and A.col_idx.tolist() == ci and A.val.tolist() == va
    pk.csr_validate(A)
    # scipy's reader (duplicates summed by tocsr) agrees, explicit zeros aside
    S = sp.csr_matrix(scipy.io.mmread(os.path.join(GOLD, name)))
    S.sum_duplicates()
    D = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(n, n))
    assert abs(S - D).max() == 0


@pytest.mark.parametrize("name", ["bad_range.mtx", "bad_count.mtx", "bad_array.mtx", "bad_rect.mtx"])
def test_rejects_malformed(name):
    with pytest.raises(ValueError):
        mtx.read_matrix_market(os.path.join(GOLD, name))


def test_rejects_skew_diagonal(tmp_path):
    f = tmp_path / "s.mtx"
    f.write_text("%%MatrixMarket matrix coordinate real skew-symmetric\n2 2 1\n1 1 3.0\n")
    with pytest.raises(ValueError):
        mtx.read_matrix_market(str(f))


def test_roundtrip_bitwise(tmp_path):
    """A generated matrix written and read back: every value bit for bit."""
    import synthgen as g
    A = g.problem("rand_1m", scale=3000).A
    f = tmp_path / "r.mtx"
    mtx.write_matrix_market(str(f), A, comment="seeded random unsymmetric, n = 3000")
    B = mtx.read_matrix_market(str(f))
    assert B.n == A.n
    assert np.array_equal(B.row_ptr, A.row_ptr) and np.array_equal(B.col_idx, A.col_idx)
    assert np.array_equal(B.val.view(np.uint64), A.val.view(np.uint64))


def test_gzip_and_stream(tmp_path):
    import gzip
    import io
    src = open(os.path.join(GOLD, "symmetric.mtx")).read()
    gz = tmp_path / "s.mtx.gz"
    with gzip.open(gz, "wt") as fh:
        fh.write(src)
    a = mtx.read_matrix_market(str(gz))
    b = mtx.read_matrix_market(io.StringIO(src))
    assert a.val.tolist() == b.val.tolist() == EXPECT["symmetric.mtx"][3]


@pytest.mark.gpu
def test_table1_runner_on_written_matrix(tmp_path):
    """The Table 1 runner on a matrix written to a .mtx file: every method converges and
    the exact-dot run matches the oracle's iteration count (b = A 1, x0 = 0)."""
    import synthgen as g
    from oracle import ctier
    from oracle.spmv import spmv
    from paper_2404_13216_amd import table1
    A = g.problem("cd2d_64", scale=24).A
    f = tmp_path / "cd2d_24.mtx"
    mtx.write_matrix_market(str(f), A)
    row = table1.run_matrix(str(f), tols=(1e-6, 1e-9), rr=50)
    assert all(v["status"] == 0 for v in row["runs"].values()), row
    ref = ctier.pbicgstab(A, spmv(A, np.ones(A.n)), tol=1e-9)
    assert row["runs"]["p-BiCGStab+exact@1e-09"]["iterations"] == ref["iterations"]
