"""Pins of the FP32 pieces of the refinement solver and of the solver itself.

* The compensated FP32 SpMV (Dot2 of Ogita, Rump and Oishi) stays within that
  algorithm's published bound |res - a.x| <= u |a.x| + gamma_n^2 sum |a_k x_k| of the
  exact rational row sum, recovers rows whose plain FP32 sum cancels to garbage, and
  agrees with a loop transcription that takes the product error from exact rational
  arithmetic.
* The plain FP32 dot (its definition: products rounded to float32, added left to right)
  is exact on small integers, obeys the worst-case gamma_n bound, and its association
  order and product rounding are pinned by
  hand-worked inputs whose result depends on that order.
* The refinement reaches the true relative residual 1e-10 with the FP64 oracle's
  solution, on every workload family; degenerate right-hand sides and the FP64
  finish behave as documented.
"""
from fractions import Fraction

import numpy as np
import pytest

import synthgen as g
from oracle import solvers
from oracle.spmv import spmv_f32, spmv_f32_loops

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1 - n * U32)


def csr_rows(rows):
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    ci, va = [], []
    for i, row in enumerate(rows):
        rp[i + 1] = rp[i] + len(row)
        for c, a in row:
            ci.append(c)
            va.append(a)
    n = max(len(rows), max(ci) + 1 if ci else 0)
    return g.CSR(len(rows), rp, np.array(ci, dtype=np.int32), np.array(va, dtype=np.float32))


def test_dot2_spmv_bound_random():
    rng = np.random.default_rng(0)
    n = 300
    rows = []
    for i in range(n):
        k = int(rng.integers(1, 40))
        cols = np.sort(rng.choice(n, k, replace=False))
        rows.append([(int(c), float(np.float32(rng.standard_normal() * 10.0 ** rng.integers(-3, 4)))) for c in cols])
    A = csr_rows(rows)
    x = (rng.standard_normal(n) * 10.0 ** rng.integers(-2, 3, n)).astype(np.float32)
    y = spmv_f32(A, x)
    for i in range(n):
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        terms = [Fraction(float(A.val[k])) * Fraction(float(x[A.col_idx[k]])) for k in range(lo, hi)]
        exact = sum(terms, Fraction(0))
        mag = sum((abs(t) for t in terms), Fraction(0))
        k = hi - lo
        assert abs(Fraction(float(y[i])) - exact) <= Fraction(U32) * abs(exact) + Fraction(gamma(k) ** 2) * mag


def test_dot2_spmv_recovers_cancellation():
    """Row terms 2^24, 1, -2^24 in that order: the plain FP32 left-to-right sum loses the
    1 (2^24 + 1 rounds to 2^24) and returns 0; Dot2 carries it and returns 1."""
    big = float(2 ** 24)
    A = csr_rows([[(0, 1.0), (1, 1.0), (2, 1.0)]])
    x = np.array([big, 1.0, -big], dtype=np.float32)
    y = spmv_f32(A, x)
    assert y[0] == np.float32(1.0)
    assert np.float32(np.float32(big) + np.float32(1.0)) - np.float32(big) == 0.0
    # products with rounding errors: (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24, minus (1 + 2^-11)
    A = csr_rows([[(0, 1.0 + 2.0 ** -12), (1, 1.0)]])
    x = np.array([1.0 + 2.0 ** -12, -(1.0 + 2.0 ** -11)], dtype=np.float32)
    y = spmv_f32(A, x)
    assert y[0] == np.float32(2.0 ** -24)          # plain FP32 gives 0: the product rounds away 2^-24
    plain = np.float32(np.float32(1.0 + 2.0 ** -12) * np.float32(1.0 + 2.0 ** -12)) - np.float32(1.0 + 2.0 ** -11)
    assert plain == 0.0


def test_dot2_spmv_matches_loops_and_empty_rows():
    p = g.problem("rand_1m", scale=4000)
    A32 = g.CSR(p.A.n, p.A.row_ptr, p.A.col_idx, p.A.val.astype(np.float32))
    x = np.random.default_rng(1).uniform(-1, 1, p.A.n).astype(np.float32)
    assert np.array_equal(spmv_f32(A32, x), np.array(spmv_f32_loops(A32, x), dtype=np.float32))
    E = csr_rows([[], [(0, 3.0)], []])
    y = spmv_f32(E, np.array([2.0], dtype=np.float32))
    assert y.tolist() == [0.0, 6.0, 0.0] and not np.signbit(y[0])


@pytest.mark.parametrize("n", [0, 1, 63, 64, 513, 4096, 4097, 70000, 2_200_000])
def test_seq_dot_exact_on_integers(n):
    rng = np.random.default_rng(n)
    a = rng.integers(-7, 8, n).astype(np.float32)
    b = rng.integers(-7, 8, n).astype(np.float32)
    exact = int(np.dot(a.astype(np.int64), b.astype(np.int64)))
    # every partial sum stays below 2^24 in magnitude, so each addition is exact
    assert np.abs(np.cumsum(a.astype(np.int64) * b.astype(np.int64))).max(initial=0) < 2 ** 24
    assert solvers.dot_f32_seq(a, b) == np.float32(exact)


@pytest.mark.parametrize("n", [1000, 50000, 300000])
def test_seq_dot_bound(n):
    rng = np.random.default_rng(n + 1)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    exact = np.dot(a.astype(np.float64), b.astype(np.float64))   # products of floats are exact in double
    err = abs(float(solvers.dot_f32_seq(a, b)) - exact)
    assert err <= gamma(n) * float(np.dot(np.abs(a).astype(np.float64), np.abs(b).astype(np.float64)))


def test_seq_dot_association_and_rounding():
    big = np.float32(2 ** 24)
    one = np.float32(1.0)
    ones = np.ones(4, dtype=np.float32)
    # left to right: (2^24 + 1) ties to 2^24, then + 1 again, then - 2^24 -> 0
    # (a pairwise order would give (2^24 + 1) + (1 - 2^24) = 2^24 + (-(2^24 - 1)) = 1)
    assert solvers.dot_f32_seq(np.array([big, one, one, -big]), ones) == 0.0
    assert solvers.dot_f32_seq(np.array([big, -big, one, one]), ones) == 2.0
    # 16 terms: numpy's own reduction would keep 8 strided partial sums and pair them,
    # (2^24 + 1) + (1 - 2^24) = 1; the sequential definition still gives 0
    a16 = np.zeros(16, dtype=np.float32)
    a16[:4] = [big, one, one, -big]
    assert solvers.dot_f32_seq(a16, np.ones(16, dtype=np.float32)) == 0.0
    # a reversed order would cancel first: 1 + 1 + (-2^24) + 2^24 -> (2 - 2^24) + 2^24 = 2
    assert solvers.dot_f32_seq(np.array([big, one, one, -big])[::-1].copy(), ones) == 2.0
    # each product is rounded to float32 before the addition: (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24
    # rounds to 1 + 2^-11 (ties to even), and the exact remainder 2^-24 is lost
    u = np.float32(1.0 + 2.0 ** -12)
    a = np.array([u, np.float32(-(1.0 + 2.0 ** -11))], dtype=np.float32)
    b = np.array([u, one], dtype=np.float32)
    assert solvers.dot_f32_seq(a, b) == 0.0
    assert solvers.dot_f32_seq(np.zeros(0, np.float32), np.zeros(0, np.float32)) == 0.0


@pytest.mark.parametrize("name,scale", [("cd2d_64", 20), ("cd2d_64", None), ("cd3d_128", 24),
                                        ("cd3d_256_var", 20), ("rand_1m", 8000)])
def test_refinement_reaches_1e10(name, scale):
    p = g.problem(name, scale=scale)
    r = solvers.ir_solve(p.A, p.b, tol=1e-10)
    assert r.status == solvers.OK and r.true_relres <= 1e-10 and r.fell_back == 0
    if name == "rand_1m":   # strongly diagonally dominant (cond ~ 10): an FP64 solve to 1e-10
        from oracle import ctier
        ref, bound = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=5000)["x"], 1e-8
    else:                   # direct solve: error ~ cond(A) u
        from scipy.sparse.linalg import spsolve
        ref, bound = spsolve(p.A.to_scipy().tocsc(), p.b), 1e-7
    assert np.linalg.norm(r.x - ref) <= bound * np.linalg.norm(ref)
    res = p.b - p.A.to_scipy() @ r.x
    assert np.linalg.norm(res) <= 1.01e-10 * np.linalg.norm(p.b)


def test_refinement_degenerate_and_finish():
    p = g.problem("cd2d_64", scale=12)
    r = solvers.ir_solve(p.A, np.zeros(p.A.n))
    assert r.status == solvers.OK and not r.x.any() and r.iterations == 0
    r = solvers.ir_solve(p.A, p.b, x0=solvers.pbicgstab(p.A, p.b, tol=1e-13).x)
    assert r.status == solvers.OK and r.iterations == 0
    bad = p.b.copy()
    bad[3] = np.nan
    assert solvers.ir_solve(p.A, bad).status == solvers.ERR_NONFINITE
    # one reliable update allowed: the FP64 finish completes the solve from the best iterate
    r = solvers.ir_solve(p.A, p.b, tol=1e-10, max_outer=1)
    assert r.fell_back == 1 and r.status == solvers.OK and r.true_relres <= 1e-10
