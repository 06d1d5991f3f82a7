"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one expression of the oracle's source on the CPU (a dropped
term, a wrong sign, a wrong index, a transposed operand, a wrong rounding) and
checks that the corresponding pin then fails.  The oracle files are not touched.
"""
import inspect
import math
import textwrap

import numpy as np
import pytest

from oracle import exact, rational, solvers
from tests.test_oracle_solvers import small_unsym


def _mutant(func, old, new):
    src = textwrap.dedent(inspect.getsource(func))
    assert old in src, old
    ns = dict(func.__globals__)
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns[func.__name__]


def _tracks_rational(pb):
    for seed in range(4):
        A, D, b = small_unsym(seed, n=8, diag=12.0)
        xs = rational.pbicgstab_q(A, b, 3)
        res = pb(A, b, tol=0.0, max_iter=len(xs), record=len(xs))
        if len(res.iterates) != len(xs):
            return False
        for (xf, _, _, _), xq in zip(res.iterates, xs):
            xq = np.array([float(v) for v in xq])
            if not np.linalg.norm(xf - xq) <= 1e-12 * np.linalg.norm(xq):
                return False
    return True


MUTATIONS = [
    ("(rw + beta * rs)", "(rw + beta * rz)"),            # wrong index
    ("r = q - omega * yv", "r = q + omega * yv"),       # wrong sign
    ("z = t + beta * (z - omega * v)", "z = t + beta * z"),  # dropped term
    ("beta = ((alpha / omega) * rho_new) / rho", "beta = ((omega / alpha) * rho_new) / rho"),  # transposed
    ("y = (y + alpha * p) + omega * q", "y = (y + alpha * p) + omega * p"),  # wrong operand
    ("w = yv - omega * (t - alpha * v)", "w = yv - omega * t"),  # dropped term
]


def test_unmutated_oracle_passes():
    assert _tracks_rational(solvers.pbicgstab)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_mutated_pbicgstab_is_caught(old, new):
    assert not _tracks_rational(_mutant(solvers.pbicgstab, old, new))


def test_mutated_rounding_is_caught():
    trunc = _mutant(exact.round_scaled, "return S / (1 << SCALE)",
                    "return float(S >> SCALE) if S > 0 else -float((-S) >> SCALE)")
    # tie case 1 + 2^-53 and a subnormal case
    assert trunc((1 << exact.SCALE) + (1 << (exact.SCALE - 53)) + 1) != 1.0 + 2.0 ** -52


def test_mutated_product_scale_is_caught():
    bad = _mutant(exact.scaled_product, "sh = ea + eb + SCALE", "sh = ea + eb + SCALE - 1")
    good = exact.scaled_product(3.0, 5.0)
    assert exact.round_scaled(bad(3.0, 5.0)) != exact.round_scaled(good)
    assert math.isclose(exact.round_scaled(good), 15.0)


# --- FP32 pieces of the refinement -------------------------------------------------
def test_mutated_dot2_spmv_is_caught():
    """Dropping the product error e from the compensation loses the 2^-24 that the
    cancellation pin demands."""
    from oracle import spmv as ospmv
    from tests.test_oracle_ir import csr_rows
    A = csr_rows([[(0, 1.0 + 2.0 ** -12), (1, 1.0)]])
    x = np.array([1.0 + 2.0 ** -12, -(1.0 + 2.0 ** -11)], dtype=np.float32)
    assert ospmv.spmv_f32(A, x)[0] == np.float32(2.0 ** -24)
    bad = _mutant(ospmv.spmv_f32, "c[rows] = c[rows] + (err + e)", "c[rows] = c[rows] + err")
    assert bad(A, x)[0] != np.float32(2.0 ** -24)


@pytest.mark.parametrize("old,new", [
    ("np.add.accumulate(prod, dtype=np.float32)[-1]", "np.add.accumulate(prod[::-1], dtype=np.float32)[-1]"),
    ("np.add.accumulate(prod, dtype=np.float32)[-1]", "np.add.reduce(prod, dtype=np.float32)"),   # pairwise
    ("np.add.accumulate(prod, dtype=np.float32)[-1]", "np.add.accumulate(prod.astype(np.float64))[-1]"),  # double sums
    ("prod = (np.asarray(a).astype(np.float32) * np.asarray(b).astype(np.float32)).astype(np.float32)\n",
     "prod = np.asarray(a).astype(np.float64) * np.asarray(b).astype(np.float64)\n"
     "    prod = prod.astype(np.float32) if prod.size < 2 else np.concatenate("
     "[(prod[:1] + prod[1:2]).astype(np.float32), np.zeros(prod.size - 1, np.float32)])\n"),  # fused first products
])
def test_mutated_seq_dot_is_caught(old, new):
    """Each planted change of the plain FP32 dot's definition fails its order / rounding pin."""
    from tests.test_oracle_ir import test_seq_dot_association_and_rounding
    test_seq_dot_association_and_rounding()
    bad = _mutant(solvers.dot_f32_seq, old, new)
    saved = solvers.dot_f32_seq
    try:
        solvers.dot_f32_seq = bad
        with pytest.raises(AssertionError):
            test_seq_dot_association_and_rounding()
    finally:
        solvers.dot_f32_seq = saved


@pytest.mark.parametrize("old,new", [
    ("        r = (r64 / nu).astype(f)\n", "        r = r if p is not None else (r64 / nu).astype(f)\n"),  # no replacement
    ("x = x + nu * d.astype(np.float64)", "x = x - nu * d.astype(np.float64)"),                          # wrong sign
])
def test_mutated_refinement_is_caught(old, new):
    import synthgen as g
    p = g.problem("cd3d_128", scale=16)
    ok = solvers.ir_solve(p.A, p.b, tol=1e-10)
    assert ok.status == solvers.OK and ok.fell_back == 0
    bad = _mutant(solvers.ir_solve, old, new)(p.A, p.b, tol=1e-10)
    assert bad.fell_back == 1 or bad.status != solvers.OK


@pytest.mark.parametrize("old,new", [
    ("vals = [float(b[i])] + (-np.asarray(A.val[a:e], dtype=np.float64)).tolist()",
     "vals = [float(b[i])] + (np.asarray(A.val[a:e], dtype=np.float64)).tolist()"),        # wrong sign
    ("xs = [1.0] + x[A.col_idx[a:e]].tolist()", "xs = [0.0] + x[A.col_idx[a:e]].tolist()"),  # b dropped
])
def test_mutated_exact_residual_is_caught(old, new):
    from oracle import spmv as ospmv
    from tests.test_oracle_exact_rows import test_brute_force_rational
    test_brute_force_rational(0)
    bad = _mutant(ospmv.resid_exact, old, new)
    saved = ospmv.resid_exact
    try:
        import tests.test_oracle_exact_rows as t
        t.resid_exact = bad
        with pytest.raises(AssertionError):
            t.test_brute_force_rational(0)
    finally:
        import tests.test_oracle_exact_rows as t
        t.resid_exact = saved


def test_mutated_exact_rows_is_caught():
    """Summing a row in floating point instead of exactly fails the cancellation pin."""
    from oracle import spmv as ospmv
    import tests.test_oracle_exact_rows as t
    t.test_cancellation_and_order_independence()
    saved = t.spmv_exact
    try:
        t.spmv_exact = lambda A, x, rows=None: ospmv.spmv(A, x)
        with pytest.raises(AssertionError):
            t.test_cancellation_and_order_independence()
    finally:
        t.spmv_exact = saved
