"""Oracle: right preconditioning and the fallback to the unpreconditioned solver.

Pins: Jacobi with a constant diagonal reproduces the unpreconditioned solve up to
scaling (in test_oracle_solvers); M = 0 makes w0 = A M r0 = 0, a breakdown at
initialisation, after which the fallback must converge from x0 = 0 exactly as the
plain solver does; a stall window triggers the fallback on a preconditioner that
stops making progress, and the true residual decides the restart point.
"""
import numpy as np

import synthgen as g
from oracle import solvers


def diag_csr(vals):
    n = len(vals)
    return g.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(vals, float))


def test_zero_preconditioner_falls_back_to_plain_solve():
    p = g.problem("cd3d_256_var", scale=12)
    M = diag_csr(np.zeros(p.A.n))
    r = solvers.pbicgstab_fallback(p.A, p.b, M, tol=1e-10)
    plain = solvers.pbicgstab(p.A, p.b, x0=np.zeros(p.A.n), tol=1e-10)
    assert r.fell_back == 1 and r.status == solvers.OK
    assert r.iterations == plain.iterations  # the preconditioned run broke down at init
    assert np.array_equal(r.x, plain.x)


def test_jacobi_no_fallback_and_fewer_iterations_on_variable_coefficients():
    p = g.problem("cd3d_256_var", scale=14)
    J = diag_csr(1.0 / p.A.diag())
    r = solvers.pbicgstab_fallback(p.A, p.b, J, tol=1e-10)
    plain = solvers.pbicgstab(p.A, p.b, tol=1e-10)
    assert r.fell_back == 0 and r.status == solvers.OK and r.true_relres <= 1e-10
    assert r.iterations < plain.iterations


def test_stall_triggers_fallback_and_true_residual_decides():
    p = g.problem("cd2d_64", scale=20)
    rng = np.random.default_rng(3)
    bad = diag_csr(rng.choice([-1.0, 1.0], p.A.n) * rng.uniform(0.01, 1.0, p.A.n))
    r1 = solvers.pbicgstab(p.A, p.b, tol=1e-10, M=bad, stall_window=5)
    r = solvers.pbicgstab_fallback(p.A, p.b, bad, tol=1e-10, stall_window=5)
    assert r.status == solvers.OK and r.true_relres <= 1e-10
    if r1.status in (solvers.STALLED, solvers.BREAKDOWN, solvers.ERR_NONFINITE):
        assert r.fell_back == 1 and r.iterations > r1.iterations
    else:
        assert r.fell_back == 0
