"""Invariants of the seeded synthetic workloads (they stand in for the paper's
SuiteSparse matrices, which are not available)."""
import math

import numpy as np
import pytest

import synthgen as g


@pytest.mark.parametrize("N", [3, 8, 31, 64])
def test_nnz_closed_forms(N):
    A2 = g.cd_stencil(N, 2, (20.0, 10.0))
    assert A2.nnz == 5 * N * N - 4 * N
    A3 = g.cd_stencil(N, 3, (30.0, 20.0, 10.0))
    assert A3.nnz == 7 * N ** 3 - 6 * N * N


def test_named_sizes():
    assert g.problem("cd2d_64").A.nnz == 20224
    # 128^3: 7n - 6N^2 = 14,581,760 (checked by formula on the small instance family)
    assert 7 * 128 ** 3 - 6 * 128 ** 2 == 14_581_760
    assert 7 * 256 ** 3 - 6 * 256 ** 2 == 117_047_296


@pytest.mark.parametrize("kappa", [False, True])
def test_stencil_structure(kappa):
    N = 10
    rng = np.random.default_rng(0)
    kap = np.exp(rng.standard_normal((N, N, N))) if kappa else None
    A = g.cd_stencil(N, 3, (5.0, -3.0, 2.0), kap)
    rp = A.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    # columns sorted ascending in each row and in range
    for i in range(A.n):
        c = A.col_idx[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and c[0] >= 0 and c[-1] < A.n
    diag = rows == A.col_idx
    assert np.all(A.val[diag] > 0) and np.all(A.val[~diag] < 0)  # M-matrix sign pattern
    rowsum = np.bincount(rows, weights=A.val, minlength=A.n)
    full = np.diff(rp) == 7  # interior rows: all neighbours present -> row sum 0
    dg = A.val[diag]
    assert np.all(np.abs(rowsum[full]) <= 16 * np.finfo(float).eps * dg[full])
    assert np.all(rowsum[~full] > 0)  # Dirichlet rows are strictly dominant


def test_upwind_values_constant():
    N, h = 4, 1.0 / 5
    A = g.cd_stencil(N, 2, (20.0, 10.0))
    # interior node (1,1) -> index 5: neighbours 1 (j-1), 4 (i-1), 6 (i+1), 9 (j+1)
    i = 5
    a, b = A.row_ptr[i], A.row_ptr[i + 1]
    cols = list(A.col_idx[a:b])
    vals = dict(zip(cols, A.val[a:b]))
    assert cols == [1, 4, 5, 6, 9]
    assert vals[4] == -1.0 - h * 20.0 and vals[6] == -1.0
    assert vals[1] == -1.0 - h * 10.0 and vals[9] == -1.0
    assert vals[5] == 4.0 + h * 30.0


def test_random_family():
    p = g.problem("rand_1m", scale=4000)
    A = p.A
    rp = A.row_ptr.astype(np.int64)
    lens = np.diff(rp)
    assert lens.min() >= 3 and lens.max() <= 401
    rows = np.repeat(np.arange(A.n), lens)
    dg = rows == A.col_idx
    assert dg.sum() == A.n
    for i in range(0, A.n, 97):
        a, b = rp[i], rp[i + 1]
        off = A.val[a:b][A.col_idx[a:b] != i]
        d = A.val[a:b][A.col_idx[a:b] == i][0]
        assert d == 1.2 * math.fsum(np.abs(off).tolist())
        assert np.all(np.diff(A.col_idx[a:b]) > 0)
    mean_off = (lens - 1).mean()
    assert 13.0 < mean_off < 20.0  # E[clip(rint(lognormal(ln 14, 0.6)))] ~ 16.8


def test_determinism():
    a = g.problem("spai_eval_128", scale=12)
    b = g.problem("spai_eval_128", scale=12)
    assert np.array_equal(a.A.val, b.A.val) and np.array_equal(a.xstar, b.xstar)
    assert np.array_equal(a.b, b.b)
    assert abs(np.linalg.norm(a.meta["velocity"]) - 50.0) < 1e-12


def test_training_params_ranges():
    for s in range(100, 300, 7):
        p = g.training_params(s)
        assert p["dim"] in (2, 3)
        n = p["N"] ** p["dim"]
        assert 0.7 * 16384 <= n <= 1.3 * 262144
        assert 1.0 <= p["peclet"] <= 100.0
