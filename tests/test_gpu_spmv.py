"""GPU CSR SpMV vs the oracle.

The default kernel (row-sequential) sums each row left to right exactly like the
oracle and must be bit-identical to it.  The vector-CSR and wavefront-per-row kernels
sum in a fixed tree order; every row must satisfy the classical bound
|y_gpu - y_oracle| <= 2 gamma_k sum_j |a_ij x_j| (Higham, Accuracy and Stability of
Numerical Algorithms, 3.1), and every kernel is bitwise identical run to run.
"""
import numpy as np
import pytest

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier
from oracle.spmv import spmv, spmv_abs
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def check_bound(A, x, y, rows=None, u=U):
    ref = spmv(A, x) if rows is None else None
    absr = spmv_abs(A, x)
    lens = np.diff(A.row_ptr.astype(np.int64))
    k = np.maximum(lens, 1)
    gam = (k * u) / (1 - k * u)
    if ref is None:
        ref = spmv(A, x)
    # oracle row value itself is within gamma_k of exact: allow both errors
    err = np.abs(y - ref)
    bound = 2 * gam * absr * (1 + 1e-12) + 1e-300
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (bad[:5], err[bad[:5]], bound[bad[:5]])


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 20), ("rand_1m", 50000),
                                        ("cd3d_256_var", 17), ("spai_eval_128", 9)])
def test_spmv_bound_and_determinism(name, scale):
    p = g.problem(name, scale=scale)
    A = pk.CSR.from_host(p.A)
    x = np.random.default_rng(1).uniform(-1, 1, p.A.n)
    tx = to_dev(x)
    ref = spmv(p.A, x)
    y = pk.csr_spmv(A, tx).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))
    for kind in (pk.SPMV_VECTOR, pk.SPMV_WAVE):
        y1 = pk.csr_spmv(A, tx, kind=kind).cpu().numpy()
        y2 = pk.csr_spmv(A, tx, kind=kind).cpu().numpy()
        assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
        check_bound(p.A, x, y1)


def test_spmv_exact_on_integers():
    """Integer-valued stencil and vector: every partial sum is exact, so any order agrees."""
    A = g.cd_stencil(30, 3, (0.0, 0.0, 0.0))
    x = np.random.default_rng(2).integers(-1000, 1000, A.n).astype(np.float64)
    y = pk.csr_spmv(pk.CSR.from_host(A), to_dev(x)).cpu().numpy()
    assert np.array_equal(y, spmv(A, x))


def test_spmv_full_size_128():
    """128^3 (2,097,152 rows, 14,581,760 nnz) at full size, checked on sampled rows."""
    p = g.problem("cd3d_128")
    A = pk.CSR.from_host(p.A)
    x = np.random.default_rng(5).uniform(-1, 1, p.A.n)
    ref = ctier.spmv(p.A, x)
    y = pk.csr_spmv(A, to_dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))
    y = pk.csr_spmv(A, to_dev(x), kind=pk.SPMV_VECTOR).cpu().numpy()
    err = np.abs(y - ref)
    absv = np.abs(p.A.val)
    rows = np.repeat(np.arange(p.A.n), np.diff(p.A.row_ptr))
    absr = np.bincount(rows, weights=absv * np.abs(x[p.A.col_idx]), minlength=p.A.n)
    assert np.all(err <= 2 * 7 * U / (1 - 7 * U) * absr * (1 + 1e-12))
    # b = A x* of the workload matches the scipy product within the same bound
    yb = pk.csr_spmv(A, to_dev(p.xstar)).cpu().numpy()
    assert np.max(np.abs(yb - p.b)) <= 1e-13 * np.max(np.abs(p.b)) + 1e-300


def test_spmv_fp32_values_and_f32_path():
    p = g.problem("rand_1m", scale=20000)
    import torch
    A64 = pk.CSR.from_host(p.A)
    A32 = A64.with_values(A64.val.to(torch.float32))
    x = np.random.default_rng(3).uniform(-1, 1, p.A.n)
    # FP32 values, FP64 x and accumulation
    y = pk.csr_spmv(A32, to_dev(x)).cpu().numpy()
    A32h = g.CSR(p.A.n, p.A.row_ptr, p.A.col_idx, p.A.val.astype(np.float32).astype(np.float64))
    check_bound(A32h, x, y)
    assert np.array_equal(y, spmv(A32h, x))  # FP32 values are exact in FP64
    # pure FP32 path: row-sequential Dot2-compensated float32, bit-identical to the oracle
    from oracle.spmv import spmv_f32
    x32 = x.astype(np.float32)
    y32 = pk.csr_spmv_f32(A32, to_dev(x32)).cpu().numpy()
    A32o = g.CSR(p.A.n, p.A.row_ptr, p.A.col_idx, p.A.val.astype(np.float32))
    assert np.array_equal(y32.view(np.uint32), spmv_f32(A32o, x32).view(np.uint32))


def test_empty_rows_and_ragged():
    rng = np.random.default_rng(9)
    n = 1000
    lens = rng.integers(0, 40, n)
    lens[::13] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=k, replace=False)) for k in lens]).astype(np.int32)
    val = rng.standard_normal(rp[-1])
    A = g.CSR(n, rp, ci, val)
    x = rng.standard_normal(n)
    for kind in (pk.SPMV_SEQ, pk.SPMV_VECTOR, pk.SPMV_WAVE):
        y = pk.csr_spmv(pk.CSR.from_host(A), to_dev(x), kind=kind).cpu().numpy()
        assert np.all(y[lens == 0] == 0.0)
        check_bound(A, x, y)
    assert np.array_equal(pk.csr_spmv(pk.CSR.from_host(A), to_dev(x)).cpu().numpy(), spmv(A, x))


def test_long_rows_chunked_staging():
    """Rows longer than one LDS chunk (2048 entries) keep the left-to-right order."""
    rng = np.random.default_rng(4)
    n = 3000
    lens = np.full(n, 3)
    lens[[0, 7, 255, 256, 2999]] = [2999, 2500, 4000 % n, 2048, 2100]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=k, replace=False)) for k in lens]).astype(np.int32)
    A = g.CSR(n, rp, ci, rng.standard_normal(rp[-1]))
    x = rng.standard_normal(n)
    y = pk.csr_spmv(pk.CSR.from_host(A), to_dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), spmv(A, x).view(np.uint64))
