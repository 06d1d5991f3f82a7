"""Pins of the exactly rounded SpMV rows (each row one exact sum, rounded once): the
oracle's definition against brute-force rational sums, hand-worked cancellations that
the sequential row sum gets wrong, ties, and the residual form b_i - (A x)_i rounded once.
"""
from fractions import Fraction

import numpy as np
import pytest

import synthgen as g
from oracle import solvers
from oracle.spmv import resid_exact, spmv, spmv_exact


def csr_rows(rows, n=None):
    rp, ci, va = [0], [], []
    for r in rows:
        for c, v in r:
            ci.append(c)
            va.append(v)
        rp.append(len(ci))
    n = n or len(rows)
    return g.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va, dtype=np.float64))


def rn(q: Fraction) -> float:
    """Round a rational to the nearest double, ties to even (CPython's int/int division
    is correctly rounded)."""
    return q.numerator / q.denominator if q else 0.0


def test_cancellation_and_order_independence():
    A = csr_rows([[(0, 1e16), (1, 1.0), (2, -1e16)], [(0, 1.0), (1, 2.0 ** -60), (2, -1.0)]])
    x = np.ones(3)
    # sequential: 1e16 + 1 rounds to 1e16, minus 1e16 -> 0; exactly: 1
    assert spmv(A, x).tolist() == [0.0, 0.0]
    assert spmv_exact(A, x).tolist() == [1.0, 2.0 ** -60]


def test_ties_round_to_even():
    # 1 + 2^-53 lies halfway between 1 and 1 + 2^-52: ties to even gives 1;
    # 1 + 2^-52 + 2^-53 is halfway between 1 + 2^-52 and 1 + 2^-51: even is 1 + 2^-51;
    # a third tiny term decides a near-tie: 1 + 2^-53 + 2^-100 rounds up
    A = csr_rows([[(0, 1.0), (1, 2.0 ** -53)], [(0, 1.0 + 2.0 ** -52), (1, 2.0 ** -53)],
                  [(0, 1.0), (1, 2.0 ** -53), (2, 2.0 ** -100)]])
    y = spmv_exact(A, np.ones(3))
    assert y.tolist() == [1.0, 1.0 + 2.0 ** -51, 1.0 + 2.0 ** -52]


@pytest.mark.parametrize("seed", range(5))
def test_brute_force_rational(seed):
    rng = np.random.default_rng(seed)
    n = 40
    rows = []
    for i in range(n):
        k = int(rng.integers(0, 12))
        cols = sorted(rng.choice(n, size=k, replace=False).tolist())
        vals = (rng.standard_normal(k) * np.exp2(rng.integers(-40, 40, k))).tolist()
        rows.append(list(zip(cols, vals)))
    A = csr_rows(rows, n)
    x = rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))
    b = rng.standard_normal(n)
    y = spmv_exact(A, x)
    r = resid_exact(A, b, x)
    for i in range(n):
        a, e = A.row_ptr[i], A.row_ptr[i + 1]
        q = sum((Fraction(float(A.val[k])) * Fraction(float(x[A.col_idx[k]])) for k in range(a, e)), Fraction(0))
        assert y[i] == rn(q)
        assert r[i] == rn(Fraction(float(b[i])) - q)
    # the residual is rounded once, not twice: on this row b - RN(Ax) != RN(b - Ax)
    B = csr_rows([[(0, 1.0), (1, 2.0 ** -53)]])
    assert resid_exact(B, np.array([1.0]), np.ones(2))[0] == -(2.0 ** -53)
    assert (np.array([1.0]) - spmv_exact(B, np.ones(2)))[0] == 0.0


def test_empty_rows_and_exact_rows_solve():
    A = csr_rows([[], [(1, 2.0)]])
    y = spmv_exact(A, np.array([3.0, 4.0]))
    assert y.tolist() == [0.0, 8.0] and not np.signbit(y[0])
    # a solve whose every A.v and residual rounds each row once converges like the
    # row-sequential one on a well-conditioned system
    p = g.problem("cd2d_64", scale=12)
    ex = solvers.default_dot(p.A.n)
    r1 = solvers.pbicgstab(p.A, p.b, tol=1e-10, dot=ex, spmv=spmv_exact,
                           resid=lambda A_, b_, x_: resid_exact(A_, b_, x_))
    r0 = solvers.pbicgstab(p.A, p.b, tol=1e-10, dot=ex)
    assert r1.status == solvers.OK and abs(r1.iterations - r0.iterations) <= 2
    assert np.linalg.norm(r1.x - r0.x) <= 1e-8 * np.linalg.norm(r0.x)
