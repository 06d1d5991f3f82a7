"""Pins of the comparators for the paper's central claim: p-BiCGStab with ordinary
FP64 dots and p-BiCGStab with residual replacement.

* The ordinary FP64 dot (its definition: products rounded to double, added left to
  right) is exact on small integers, obeys the gamma_n bound, and its association order
  and product rounding are pinned by hand-worked inputs (2^53 + 1 rounds to 2^53).
* Residual replacement does not change the iterates in exact arithmetic, so the FP64
  run with replacement must still track the rational Algorithm 2 (as the plain run
  does); a planted mistake in the replacement is caught by the same check.
* The ordinary-dot run tracks the rational iterates too (its dots differ from exact by
  a few ulps), and passing the exact dot in its place reproduces the exact run bit for
  bit (the plumbing of recurrence dots vs. the exact ||b|| / true residual).
"""
import numpy as np
import pytest

import synthgen as g
from oracle import ctier, rational, solvers
from tests.test_oracle_mutations import _mutant
from tests.test_oracle_solvers import small_unsym

U64 = 2.0 ** -53


@pytest.mark.parametrize("n", [0, 1, 64, 4097, 70000, 1_500_000])
def test_f64_seq_dot_exact_on_integers(n):
    rng = np.random.default_rng(n + 7)
    a = rng.integers(-1000, 1001, n).astype(np.float64)
    b = rng.integers(-1000, 1001, n).astype(np.float64)
    assert solvers.dot_f64_seq(a, b) == float(np.dot(a.astype(np.int64), b.astype(np.int64)))


def test_f64_seq_dot_bound_and_order():
    rng = np.random.default_rng(3)
    n = 200000
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    exact = ctier.exact_dot(a, b)
    gam = n * U64 / (1 - n * U64)
    assert abs(solvers.dot_f64_seq(a, b) - exact) <= gam * float(np.dot(np.abs(a), np.abs(b)))
    big = 2.0 ** 53
    # left to right: 2^53 + 1 ties to 2^53 (twice), then - 2^53 -> 0; a pairwise order
    # would give 1, the reversed order 2
    assert solvers.dot_f64_seq(np.array([big, 1.0, 1.0, -big]), np.ones(4)) == 0.0
    assert solvers.dot_f64_seq(np.array([-big, 1.0, 1.0, big]), np.ones(4)) == 2.0
    # products rounded to double first: (1 + 2^-27)^2 = 1 + 2^-26 + 2^-54 -> 1 + 2^-26
    u = 1.0 + 2.0 ** -27
    assert solvers.dot_f64_seq(np.array([u, -(1.0 + 2.0 ** -26)]), np.array([u, 1.0])) == 0.0


def _tracks(kw, tol=1e-12, dot=None):
    for seed in range(4):
        A, D, b = small_unsym(seed, n=8, diag=12.0)
        xs = rational.pbicgstab_q(A, b, 6)
        res = solvers.pbicgstab(A, b, tol=0.0, max_iter=len(xs), record=len(xs), dot=dot, **kw)
        if len(res.iterates) != len(xs):
            return False
        for (xf, _, _, _), xq in zip(res.iterates, xs):
            xq = np.array([float(v) for v in xq])
            if not np.linalg.norm(xf - xq) <= tol * np.linalg.norm(xq):
                return False
    return True


@pytest.mark.parametrize("period", [1, 2, 3])
def test_replacement_tracks_rational(period):
    assert _tracks({"rr_period": period})


def test_replacement_mutation_caught():
    bad = _mutant(solvers.pbicgstab, "            z = op.apply(s)\n            v = op.apply(z)\n",
                  "            z = op.apply(p)\n            v = op.apply(z)\n")
    ok = True
    for seed in range(4):
        A, D, b = small_unsym(seed, n=8, diag=12.0)
        xs = rational.pbicgstab_q(A, b, 6)
        res = bad(A, b, tol=0.0, max_iter=len(xs), record=len(xs), rr_period=2)
        for (xf, _, _, _), xq in zip(res.iterates, xs):
            xq = np.array([float(v) for v in xq])
            ok = ok and np.linalg.norm(xf - xq) <= 1e-12 * np.linalg.norm(xq)
    assert not ok


def test_plain_dots_track_rational():
    assert _tracks({"exact_dot": None}, tol=1e-11, dot=solvers.dot_f64_seq)


def test_plain_dot_plumbing():
    """dot = exact dot in the plain slot reproduces the exact run bit for bit."""
    p = g.problem("cd2d_64", scale=24)
    ex = solvers.pbicgstab(p.A, p.b, tol=1e-10)
    same = solvers.pbicgstab(p.A, p.b, tol=1e-10, dot=solvers.default_dot(p.A.n),
                             exact_dot=solvers.default_dot(p.A.n))
    assert ex.iterations == same.iterations and np.array_equal(ex.x, same.x)
    pl = solvers.pbicgstab(p.A, p.b, tol=1e-10, dot=solvers.dot_f64_seq, exact_dot=solvers.default_dot(p.A.n))
    assert pl.status == solvers.OK and pl.true_relres <= 1e-10
    assert np.linalg.norm(pl.x - ex.x) <= 1e-8 * np.linalg.norm(ex.x)


def test_fp32_matrix_form_pins():
    """The FP32-matrix form: on a matrix whose values are exact in FP32 (integers) it is
    p-BiCGStab with residual replacement, bit for bit; on the families it reaches the true
    residual 1e-10 and the FP64 solution; a planted mistake (replacement with the FP32
    values) is caught on a matrix whose values are not exact in FP32."""
    from synthgen import CSR
    p = g.problem("cd2d_64", scale=20)
    Ai = CSR(p.A.n, p.A.row_ptr, p.A.col_idx, np.rint(p.A.val * 4000.0))
    bi = p.b * 4000.0
    r1 = solvers.pbicgstab_fp32_matrix(Ai, bi, rr_period=7)
    r2 = solvers.pbicgstab(Ai, bi, rr_period=7, dot=solvers.default_dot(Ai.n))
    assert r1.iterations == r2.iterations and np.array_equal(r1.x.view(np.uint64), r2.x.view(np.uint64))
    for name, scale in (("cd3d_256_var", 20), ("rand_1m", 4000), ("cd3d_128", 24)):
        q = g.problem(name, scale=scale)
        r = solvers.pbicgstab_fp32_matrix(q.A, q.b)
        ref = ctier.bicgstab(q.A, q.b, tol=1e-10)
        assert r.status == solvers.OK and r.true_relres <= 1e-10
        assert np.linalg.norm(r.x - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
    q = g.problem("cd3d_256_var", scale=20)
    bad = _mutant(solvers.pbicgstab_fp32_matrix, "resid=lambda _A, b_, x_: b_ - _spmv(A, x_)",
                  "resid=lambda _A, b_, x_: b_ - _spmv(A32, x_)")(q.A, q.b)
    # replacing with the FP32 matrix solves fp32(A) x = b: measured against the FP64 A its
    # residual stays far above the tolerance
    from oracle.spmv import spmv
    res = q.b - spmv(q.A, bad.x)
    assert np.sqrt(ctier.exact_dot(res, res) / ctier.exact_dot(q.b, q.b)) > 1e-9
