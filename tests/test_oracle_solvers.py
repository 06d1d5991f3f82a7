"""Pins of the oracle's SpMV, BiCGStab (Algorithm 1) and p-BiCGStab (Algorithm 2).

Pins: rational BiCGStab == rational p-BiCGStab iterate by iterate (the paper's
mathematical-equivalence statement, Section 2); finite termination in exact
arithmetic; dense LU solutions; closed-form special cases (A = I lucky
breakdown, skew-symmetric breakdown at initialisation, diagonal matrices with k
distinct eigenvalues); scipy's CSR mat-vec and plain Python loops for SpMV; the
two oracle tiers bit-identical.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import synthgen as g
from oracle import ctier, rational, solvers
from oracle.spmv import spmv, spmv_loops


def csr_from_dense(D):
    S = sp.csr_matrix(D)
    S.sort_indices()
    return g.CSR(D.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


def small_unsym(seed, n=6, lo=-3, hi=4, diag=8.0):
    rng = np.random.default_rng(seed)
    D = rng.integers(lo, hi, (n, n)).astype(float) + np.diag(np.full(n, diag))
    D[rng.random((n, n)) < 0.3] = 0.0
    np.fill_diagonal(D, diag + rng.integers(0, 3, n))
    b = rng.integers(-5, 6, n).astype(float)
    if not b.any():
        b[0] = 1.0
    return csr_from_dense(D), D, b


# ---------------------------------------------------------------- SpMV
def test_spmv_matches_loops_and_scipy():
    p = g.problem("cd2d_64", scale=12)
    x = np.random.default_rng(0).standard_normal(p.A.n)
    y = spmv(p.A, x)
    assert np.array_equal(y, np.array(spmv_loops(p.A, x)))
    assert np.array_equal(y, p.A.to_scipy() @ x)  # scipy sums rows left to right
    assert np.array_equal(y, ctier.spmv(p.A, x))
    r = g.problem("rand_1m", scale=3000)
    x = np.random.default_rng(1).standard_normal(r.A.n)
    assert np.array_equal(spmv(r.A, x), r.A.to_scipy() @ x)
    assert np.array_equal(spmv(r.A, x), ctier.spmv(r.A, x))


def test_spmv_rows_within_higham_bound():
    """|y - RN(exact row)| <= gamma_len * sum |a x| (Higham, Accuracy and Stability, 3.1)."""
    from oracle.exact import exact_dot
    r = g.problem("rand_1m", scale=500)
    A = r.A
    x = np.random.default_rng(3).standard_normal(A.n)
    y = spmv(A, x)
    u = 2.0 ** -53
    for i in range(0, A.n, 7):
        a, b = int(A.row_ptr[i]), int(A.row_ptr[i + 1])
        ex = exact_dot(A.val[a:b].tolist(), x[A.col_idx[a:b]].tolist())
        k = b - a
        gam = k * u / (1 - k * u)
        assert abs(y[i] - ex) <= gam * float(np.sum(np.abs(A.val[a:b] * x[A.col_idx[a:b]]))) * (1 + 1e-12)


# ---------------------------------------------------------------- rational pins
@pytest.mark.parametrize("seed", range(8))
def test_rational_bicgstab_equals_pbicgstab(seed):
    A, D, b = small_unsym(seed)
    xb = rational.bicgstab_q(A, b, 8)
    xp = rational.pbicgstab_q(A, b, 8)
    assert len(xb) == len(xp) and len(xb) >= 1
    for u, v in zip(xb, xp):
        assert u == v


@pytest.mark.parametrize("seed", range(5))
def test_rational_finite_termination(seed):
    A, D, b = small_unsym(seed, n=5)
    xs = rational.pbicgstab_q(A, b, 10)
    M = rational._dense(A)
    res = [Fraction(float(bi)) - s for bi, s in zip(b, rational._mv(M, xs[-1]))]
    assert len(xs) <= A.n and all(v == 0 for v in res)


@pytest.mark.parametrize("seed", range(4))
def test_fp64_oracle_tracks_rational(seed):
    """FP64 iterates equal the exact ones up to rounding in the first iterations."""
    A, D, b = small_unsym(seed, n=8, diag=12.0)
    xs = rational.pbicgstab_q(A, b, 3)
    res = solvers.pbicgstab(A, b, tol=0.0, max_iter=len(xs), record=len(xs))
    for (xf, _, _, _), xq in zip(res.iterates, xs):
        xq = np.array([float(v) for v in xq])
        assert np.linalg.norm(xf - xq) <= 1e-12 * np.linalg.norm(xq)


# ---------------------------------------------------------------- FP64 solvers
@pytest.mark.parametrize("alg", ["p", "b"])
@pytest.mark.parametrize("seed", range(4))
def test_lu_agreement(alg, seed):
    rng = np.random.default_rng(seed)
    n = 40
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.2) + np.diag(rng.uniform(4, 8, n))
    A = csr_from_dense(D)
    b = rng.standard_normal(n)
    f = solvers.pbicgstab if alg == "p" else solvers.bicgstab
    r = f(A, b, tol=1e-12, max_iter=500)
    xl = np.linalg.solve(D, b)
    assert r.status == solvers.OK and r.true_relres <= 1e-12
    assert np.linalg.norm(r.x - xl) <= 1e-9 * np.linalg.norm(xl)


@pytest.mark.parametrize("alg", ["p", "b"])
def test_identity_lucky_breakdown(alg):
    n = 17
    A = csr_from_dense(np.eye(n))
    b = np.random.default_rng(0).standard_normal(n)
    f = solvers.pbicgstab if alg == "p" else solvers.bicgstab
    r = f(A, b, tol=1e-10)
    assert r.status == solvers.OK and r.iterations == 1
    assert np.array_equal(r.x, b)


def test_skew_symmetric_breakdown_at_init():
    """(r0, A r0) = 0 exactly for skew-symmetric A: p-BiCGStab cannot start."""
    rng = np.random.default_rng(1)
    n = 12
    K = np.triu(rng.integers(-4, 5, (n, n)).astype(float), 1)
    K = K - K.T
    A = csr_from_dense(K)
    b = rng.integers(-3, 4, n).astype(float)
    r = solvers.pbicgstab(A, b, tol=1e-10)
    assert r.status == solvers.BREAKDOWN and r.iterations == 0
    assert ctier.pbicgstab(A, b)["status"] == solvers.BREAKDOWN


@pytest.mark.parametrize("k", [1, 2, 3])
def test_diagonal_k_eigenvalues(k):
    n = 30
    ev = np.array([2.0, 5.0, 11.0])[:k]
    D = np.diag(np.resize(ev, n))
    A = csr_from_dense(D)
    b = np.random.default_rng(k).uniform(-1, 1, n)
    r = solvers.pbicgstab(A, b, tol=1e-13, max_iter=50)
    assert r.status == solvers.OK and r.iterations <= k + 1


def test_nan_rhs_and_zero_rhs_and_tol_zero():
    A, D, b = small_unsym(0)
    bn = b.copy()
    bn[2] = math.nan
    assert solvers.pbicgstab(A, bn).status == solvers.ERR_NONFINITE
    assert ctier.pbicgstab(A, bn)["status"] == solvers.ERR_NONFINITE
    r = solvers.pbicgstab(A, np.zeros(A.n))
    assert r.status == solvers.OK and r.iterations == 0 and not r.x.any()
    p = g.problem("cd2d_64", scale=16)
    r = solvers.pbicgstab(p.A, p.b, tol=0.0, max_iter=7)
    assert r.status in (solvers.NOT_CONVERGED, solvers.BREAKDOWN) and r.iterations <= 7


@pytest.mark.parametrize("alg", ["p", "b"])
def test_tiers_bit_identical(alg):
    for name, sc in (("cd2d_64", 24), ("rand_1m", 2000)):
        p = g.problem(name, scale=sc)
        f1 = solvers.pbicgstab if alg == "p" else solvers.bicgstab
        f2 = ctier.pbicgstab if alg == "p" else ctier.bicgstab
        r1 = f1(p.A, p.b, tol=1e-10, max_iter=500)
        r2 = f2(p.A, p.b, tol=1e-10, max_iter=500, history=True)
        assert r1.status == r2["status"] == solvers.OK
        assert r1.iterations == r2["iterations"]
        assert np.array_equal(r1.x, r2["x"])
        assert np.array_equal(np.array(r1.history), r2["history"])


def test_cd2d_64_reaches_true_residual():
    p = g.problem("cd2d_64")
    r = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=2000)
    assert r["status"] == solvers.OK and r["true_relres"] <= 1e-10
    assert np.linalg.norm(r["x"] - p.xstar) <= 1e-7 * np.linalg.norm(p.xstar)


def test_right_preconditioned_jacobi_invariance():
    """With a constant diagonal d, Jacobi M = I/d only rescales the Krylov iterates."""
    p = g.problem("cd2d_64", scale=16)
    A = p.A
    dg = A.diag()
    assert np.all(dg == dg[0])
    M = g.CSR(A.n, np.arange(A.n + 1, dtype=np.int32), np.arange(A.n, dtype=np.int32),
              np.full(A.n, 1.0 / dg[0]))
    r1 = solvers.pbicgstab(A, p.b, tol=1e-10, M=M)
    r0 = solvers.pbicgstab(A, p.b, tol=1e-10)
    assert r1.status == r0.status == solvers.OK
    assert abs(r1.iterations - r0.iterations) <= 1
    assert np.linalg.norm(r1.x - r0.x) <= 1e-8 * np.linalg.norm(r0.x)


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 32), ("rand_1m", 20000)])
def test_stagnation_rule_tiers_agree(name, scale):
    """A tolerance below what p-BiCGStab's recurrences sustain (1e-14): failed true-residual
    tests, then STAGNATED well before the iteration cap with the best tested iterate --
    identically in the Python and C tiers.  BiCGStab reaches the same tolerance."""
    p = g.problem(name, scale=scale)
    dot = ctier.exact_dot   # the C tier's exact dot (bit-identical to tier 1, pinned above)
    r1 = solvers.pbicgstab(p.A, p.b, tol=1e-14, max_iter=3000, dot=dot)
    r2 = ctier.pbicgstab(p.A, p.b, tol=1e-14, max_iter=3000)
    assert r1.status == r2["status"] == solvers.STAGNATED
    assert r1.iterations == r2["iterations"] < 1000
    assert r1.true_checks == r2["true_checks"] >= 3
    assert np.array_equal(r1.x, r2["x"]) and r1.true_relres == r2["true_relres"]
    res = p.b - p.A.to_scipy() @ r1.x
    assert abs(np.linalg.norm(res) / np.linalg.norm(p.b) / r1.true_relres - 1) < 1e-6  # the returned iterate's
    b1 = solvers.bicgstab(p.A, p.b, tol=1e-14, max_iter=3000, dot=dot)
    b2 = ctier.bicgstab(p.A, p.b, tol=1e-14, max_iter=3000)
    assert b1.status == b2["status"] == solvers.OK and np.array_equal(b1.x, b2["x"])
