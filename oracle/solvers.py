"""BiCGStab (Algorithm 1) and pipelined BiCGStab (Algorithm 2) in FP64 with exact
dot products -- oracle.

Vector updates are numpy element-wise expressions in exactly the parenthesisation
below; numpy rounds every operation separately (no contraction), which is the
literal-order reading of the paper's recurrences.  All inner products go through
``dot`` (exact, rounded once); A.v goes through ``spmv`` (row-sequential).

Readings of Algorithm 2 (p-BiCGStab) where the printed text is garbled or silent:

* w_0 is A r_0 (the printed ``A - r_0`` is a typo; w_i = A r_i is the invariant
  the update of w_{i+1} and the alpha recurrence rely on);
* the scalar omega and the vector w share the symbol w in the paper; here the
  scalar is ``omega`` and the vector is ``w``;
* in iteration 0, p_{-1}, s_{-1}, z_{-1}, v_{-1}, omega_{-1} are multiplied by
  beta_{-1} = 0; they are undefined, so p_0 = r_0, s_0 = w_0, z_0 = t_0 are plain
  copies;
* the shadow residual r_hat is r_0 (every inner product in the paper is taken
  against r_0);
* beta_i = (alpha_i / omega_i) (r_hat, r_{i+1}) / (r_hat, r_i) is evaluated left to
  right: ((alpha/omega) * rho_new) / rho;
* alpha_{i+1} = rho_new / ((r_hat, w_{i+1}) + beta (r_hat, s_i) - (beta omega)(r_hat, z_i))
  is evaluated as rho_new / (((rw + beta*rs) - (beta*omega)*rz));
* x_{i+1} = x_i + alpha p_i + omega q_i is evaluated as (x + alpha*p) + omega*q.

Stopping (the paper states tolerances but not the norm): after each iteration
rec = sqrt((r, r)) / ||b||; when rec <= tol the true relative residual
sqrt((b - A x, b - A x)) / ||b|| is computed and the solve stops if it is <= tol,
otherwise it continues.  After a failed test the next one comes 5 iterations later
(whatever rec does); 30 failed tests in a row without a new smallest true residual end
the solve with STAGNATED (the recursive residual has left the true one behind),
returning the iterate of the best failed test.  ``iterations`` counts completed loop bodies.

Breakdowns (the paper is silent): ||b|| = 0 -> x = 0, OK; (r_hat, w_0) = 0 or an
alpha denominator = 0 or rho = 0 or omega = 0 -> BREAKDOWN; (y, y) = 0 and
(q, q) = 0 -> lucky breakdown: x = x + alpha p and the true residual decides;
(y, y) = 0 with q != 0 -> BREAKDOWN; any non-finite scalar -> ERR_NONFINITE.
The current iterate is always returned.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import exact
from .spmv import spmv as _spmv, spmv_f32 as _spmv_f32

OK, NOT_CONVERGED, BREAKDOWN, STAGNATED = 0, 1, 2, 3
STALLED = 4  # internal: the preconditioned solve stalled (triggers the fallback)
ERR_INVALID, ERR_HIP, ERR_NONFINITE, ERR_WORKSPACE = -1, -2, -3, -4


@dataclasses.dataclass
class Result:
    x: np.ndarray
    status: int
    iterations: int
    true_relres: float
    rec_relres: float
    true_checks: int = 0
    history: list = dataclasses.field(default_factory=list)
    iterates: list = dataclasses.field(default_factory=list)  # (x, r, alpha, omega) per iteration
    outer_iterations: int = 0
    fell_back: int = 0
    true_history: list = dataclasses.field(default_factory=list)


def default_dot(n: int):
    """Exact dot: tier 1 for small n, the bit-identical C tier for large n."""
    if n <= 20000:
        return lambda a, b: exact.exact_dot(a.tolist(), b.tolist())
    from . import ctier
    return ctier.exact_dot


def _finite(*v):
    return all(math.isfinite(t) for t in v)


class _Operator:
    """A (unpreconditioned) or A.M (right preconditioning); x = M y at the end."""

    def __init__(self, A, M, spmv):
        self.A, self.M, self.spmv = A, M, spmv

    def apply(self, v):
        if self.M is None:
            return self.spmv(self.A, v)
        return self.spmv(self.A, self.spmv(self.M, v))

    def to_x(self, y):
        return y if self.M is None else self.spmv(self.M, y)


class _TrueTest:
    """When the true residual is tested, and when failed tests mean stagnation.

    The first test comes as soon as rec <= tol; after a failed test the next comes 5
    iterations later (whatever rec does).  A failed test with a true residual below
    every earlier one keeps its iterate; 30 failed tests in a row without a new best
    mean stagnation, and the solve returns the kept iterate."""

    EVERY, PATIENCE = 5, 30

    def __init__(self, tol):
        self.tol, self.best, self.stag, self.it_fail = tol, math.inf, 0, -1
        self.x_best = None

    def due(self, rec, it):
        if self.it_fail < 0:
            return rec <= self.tol
        return it - self.it_fail >= self.EVERY

    def failed(self, rec, tr, it, x):
        """Record a failed test at iteration it with iterate x; True on stagnation."""
        self.it_fail = it
        if tr < self.best:
            self.best, self.stag, self.x_best = tr, 0, x.copy()
            return False
        self.stag += 1
        return self.stag >= self.PATIENCE


def _resid_seq(spmv):
    return lambda A, b, x: b - spmv(A, x)


def _true_relres(A, b, x, normb, dot, resid):
    res = resid(A, b, x)
    return math.sqrt(dot(res, res)) / normb


def pbicgstab(A, b, x0=None, tol=1e-10, max_iter=10000, M=None, dot=None, spmv=None,
              record=0, stall_window=0, exact_dot=None, rr_period=0, true_every=0, resid=None) -> Result:
    """p-BiCGStab, Algorithm 2, with the readings in the module docstring.

    With ``M`` (a CSR right preconditioner) the recurrences run on A.M and y,
    starting from y_0 = 0, and x = M y; ``x0`` must then be None.
    ``record`` keeps (x_i, r_i, alpha, omega) for the first ``record`` iterations.
    ``dot`` forms the inner products of the recurrences; ``exact_dot`` (default: the
    same) forms ||b||, the true residual and the (q, q) test -- with dot = dot_f64_seq
    and the exact dot there, this is the ordinary-dot comparator.
    ``rr_period`` > 0: residual replacement (the p-BiCGStabRR variant the paper refers
    to) after every rr_period-th completed iteration: r = b - A x, w = A r, t = A w,
    s = A p, z = A s, v = A z, with the scalars kept (unpreconditioned only).
    ``true_every`` > 0: after every true_every-th completed iteration the solve
    continues from, the true relative residual is appended to ``true_history``.
    ``resid(A, b, x)`` forms b - A x wherever the solve needs it (r_0, the true residual,
    replacement); default b - spmv(A, x) (two roundings per row); ``oracle.spmv.resid_exact``
    rounds each row of it once.
    """
    spmv = spmv or _spmv
    resid = resid or _resid_seq(spmv)
    n = A.n
    dot = dot or default_dot(n)
    xdot = exact_dot or dot
    if rr_period and M is not None:
        raise ValueError("residual replacement is defined for the unpreconditioned solve")
    op = _Operator(A, M, spmv)
    b = np.asarray(b, dtype=np.float64)
    if M is not None and x0 is not None:
        raise ValueError("right-preconditioned solve starts from y0 = 0")
    y = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)

    true_hist = []

    def finish(status, iters, rec, hist, its, checks, true=None):
        x = op.to_x(y)
        if true is None:
            true = _true_relres(A, b, x, normb, xdot, resid) if normb > 0 else 0.0
        return Result(x, status, iters, true, rec, checks, hist, its, true_history=true_hist)

    nb2 = xdot(b, b)
    if not math.isfinite(nb2):
        return Result(op.to_x(y), ERR_NONFINITE, 0, math.nan, math.nan)
    normb = math.sqrt(nb2)
    if normb == 0.0:
        return Result(np.zeros(n), OK, 0, 0.0, 0.0)
    # initialisation (Algorithm 2, before the loop)
    r = resid(A, b, op.to_x(y)) if x0 is not None else b.copy()
    rhat = r.copy()
    w = op.apply(r)
    t = op.apply(w)
    rho = dot(rhat, r)
    rw = dot(rhat, w)
    rec = math.sqrt(dot(r, r)) / normb
    hist, its, checks = [], [], 0
    test = _TrueTest(tol)
    if test.due(rec, 0):
        checks += 1
        tr = _true_relres(A, b, op.to_x(y), normb, xdot, resid)
        if tr <= tol:
            return finish(OK, 0, rec, hist, its, checks, tr)
        if test.failed(rec, tr, 0, y):
            y = test.x_best
            return finish(STAGNATED, 0, rec, hist, its, checks, test.best)
    if not _finite(rho, rw):
        return finish(ERR_NONFINITE, 0, rec, hist, its, checks)
    if rw == 0.0:
        return finish(BREAKDOWN, 0, rec, hist, its, checks)
    alpha = rho / rw
    beta = omega = 0.0
    p = s = z = v = None
    for i in range(max_iter):
        if i == 0:
            p, s, z = r.copy(), w.copy(), t.copy()
        else:
            p = r + beta * (p - omega * s)
            s = w + beta * (s - omega * z)
            z = t + beta * (z - omega * v)
        q = r - alpha * s
        yv = w - alpha * z
        qy = dot(q, yv)
        yy = dot(yv, yv)
        rs = dot(rhat, s)
        rz = dot(rhat, z)
        v = op.apply(z)
        if not _finite(qy, yy, rs, rz):
            return finish(ERR_NONFINITE, i, rec, hist, its, checks)
        if yy == 0.0:
            if xdot(q, q) == 0.0:  # lucky breakdown: r_{i+1} = q_i = 0
                y = y + alpha * p
                checks += 1
                tr = _true_relres(A, b, op.to_x(y), normb, xdot, resid)
                return finish(OK if tr <= tol else BREAKDOWN, i + 1, 0.0, hist, its, checks, tr)
            return finish(BREAKDOWN, i, rec, hist, its, checks)
        omega = qy / yy
        if omega == 0.0:
            return finish(BREAKDOWN, i, rec, hist, its, checks)
        y = (y + alpha * p) + omega * q
        r = q - omega * yv
        w = yv - omega * (t - alpha * v)
        t = op.apply(w)
        rho_new = dot(rhat, r)
        rw = dot(rhat, w)
        rr = dot(r, r)
        rec = math.sqrt(rr) / normb
        hist.append(rec)
        if len(its) < record:
            its.append((op.to_x(y), r.copy(), alpha, omega))
        beta = ((alpha / omega) * rho_new) / rho
        den = (rw + beta * rs) - (beta * omega) * rz
        alpha_new = rho_new / den if den != 0.0 else math.nan
        if test.due(rec, i + 1):
            checks += 1
            tr = _true_relres(A, b, op.to_x(y), normb, xdot, resid)
            if tr <= tol:
                return finish(OK, i + 1, rec, hist, its, checks, tr)
            if test.failed(rec, tr, i + 1, y):
                y = test.x_best
                return finish(STAGNATED, i + 1, rec, hist, its, checks, test.best)
        if not _finite(rho_new, rw, rr, beta) or (den != 0.0 and not math.isfinite(alpha_new)):
            return finish(ERR_NONFINITE, i + 1, rec, hist, its, checks)
        if rho_new == 0.0 or den == 0.0:
            return finish(BREAKDOWN, i + 1, rec, hist, its, checks)
        # stall: the recursive residual has not halved over the last `stall_window` iterations
        if stall_window and len(hist) > stall_window and rec > 0.5 * hist[-1 - stall_window]:
            return finish(STALLED, i + 1, rec, hist, its, checks)
        alpha, rho = alpha_new, rho_new
        if i + 1 == max_iter:          # the solve does not continue from the last iteration
            break
        if true_every and (i + 1) % true_every == 0:
            true_hist.append(_true_relres(A, b, op.to_x(y), normb, xdot, resid))
        if rr_period and (i + 1) % rr_period == 0:
            r = resid(A, b, y)
            w = op.apply(r)
            t = op.apply(w)
            s = op.apply(p)
            z = op.apply(s)
            v = op.apply(z)
    return finish(NOT_CONVERGED, max_iter, rec, hist, its, checks)


def bicgstab(A, b, x0=None, tol=1e-10, max_iter=10000, dot=None, spmv=None, record=0) -> Result:
    """BiCGStab, Algorithm 1 (van der Vorst), same dots, stopping rule and breakdowns.

    Per iteration: s = A p; alpha = rho / (r_hat, s); q = r - alpha s; y = A q;
    omega = (q, y) / (y, y); x = (x + alpha p) + omega q; r = q - omega y;
    rho' = (r_hat, r); beta = ((alpha / omega) rho') / rho; p = r + beta (p - omega s).
    """
    spmv = spmv or _spmv
    n = A.n
    dot = dot or default_dot(n)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb2 = dot(b, b)
    if not math.isfinite(nb2):
        return Result(x, ERR_NONFINITE, 0, math.nan, math.nan)
    normb = math.sqrt(nb2)
    if normb == 0.0:
        return Result(np.zeros(n), OK, 0, 0.0, 0.0)

    def finish(status, iters, rec, true=None):
        if true is None:
            true = _true_relres(A, b, x, normb, dot, _resid_seq(spmv))
        return Result(x, status, iters, true, rec, checks, hist, its)

    r = b - spmv(A, x) if x0 is not None else b.copy()
    rhat = r.copy()
    p = r.copy()
    rho = dot(rhat, r)
    rec = math.sqrt(dot(r, r)) / normb
    hist, its, checks = [], [], 0
    test = _TrueTest(tol)
    if test.due(rec, 0):
        checks += 1
        tr = _true_relres(A, b, x, normb, dot, _resid_seq(spmv))
        if tr <= tol:
            return finish(OK, 0, rec, tr)
        if test.failed(rec, tr, 0, x):
            x = test.x_best
            return finish(STAGNATED, 0, rec, test.best)
    if not math.isfinite(rho):
        return finish(ERR_NONFINITE, 0, rec)
    for i in range(max_iter):
        s = spmv(A, p)
        rs = dot(rhat, s)
        if not math.isfinite(rs):
            return finish(ERR_NONFINITE, i, rec)
        if rs == 0.0 or rho == 0.0:
            return finish(BREAKDOWN, i, rec)
        alpha = rho / rs
        q = r - alpha * s
        yv = spmv(A, q)
        qy = dot(q, yv)
        yy = dot(yv, yv)
        if not _finite(qy, yy):
            return finish(ERR_NONFINITE, i, rec)
        if yy == 0.0:
            if dot(q, q) == 0.0:
                x = x + alpha * p
                checks += 1
                tr = _true_relres(A, b, x, normb, dot, _resid_seq(spmv))
                return finish(OK if tr <= tol else BREAKDOWN, i + 1, 0.0, tr)
            return finish(BREAKDOWN, i, rec)
        omega = qy / yy
        if omega == 0.0:
            return finish(BREAKDOWN, i, rec)
        x = (x + alpha * p) + omega * q
        r = q - omega * yv
        rho_new = dot(rhat, r)
        rr = dot(r, r)
        rec = math.sqrt(rr) / normb
        hist.append(rec)
        if len(its) < record:
            its.append((x.copy(), r.copy(), alpha, omega))
        beta = ((alpha / omega) * rho_new) / rho
        if test.due(rec, i + 1):
            checks += 1
            tr = _true_relres(A, b, x, normb, dot, _resid_seq(spmv))
            if tr <= tol:
                return finish(OK, i + 1, rec, tr)
            if test.failed(rec, tr, i + 1, x):
                x = test.x_best
                return finish(STAGNATED, i + 1, rec, test.best)
        if not _finite(rho_new, rr, beta):
            return finish(ERR_NONFINITE, i + 1, rec)
        if rho_new == 0.0:
            return finish(BREAKDOWN, i + 1, rec)
        p = r + beta * (p - omega * s)
        rho = rho_new
    return finish(NOT_CONVERGED, max_iter, rec)


# ---------------------------------------------------------------------------
# FP32 inner p-BiCGStab inside FP64 iterative refinement
# ---------------------------------------------------------------------------

def dot_f32_seq(a: np.ndarray, b: np.ndarray) -> np.float32:
    """Plain float32 dot by its definition: every product a_i b_i rounded to float32 and
    added left to right, s_k = fl32(s_(k-1) + p_k) from s_0 = 0 (ufunc.accumulate is a
    strictly sequential scan) -- the inner products of the FP32 solver."""
    prod = (np.asarray(a).astype(np.float32) * np.asarray(b).astype(np.float32)).astype(np.float32)
    if prod.size == 0:
        return np.float32(0.0)
    return np.float32(np.add.accumulate(prod, dtype=np.float32)[-1])


def dot_f64_seq(a: np.ndarray, b: np.ndarray) -> float:
    """Ordinary FP64 dot by its definition: products rounded to double, added left to
    right -- the non-exact comparator of the paper's claim about exact inner products."""
    prod = np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)
    if prod.size == 0:
        return 0.0
    return float(np.add.accumulate(prod)[-1])


# reasons that end a run of FP32 iterations (bit flags)
_RU_CHECK, _RU_CONVERGED, _RU_BREAKDOWN, _RU_NONFINITE, _RU_STALL, _RU_MAXIT, _RU_YYZERO = 1, 2, 4, 8, 16, 32, 64
_RU_RESTART = _RU_BREAKDOWN | _RU_NONFINITE | _RU_STALL | _RU_YYZERO


def pbicgstab_fallback(A, b, M, tol=1e-10, max_iter=10000, stall_window=200, dot=None, spmv=None) -> Result:
    """Right-preconditioned p-BiCGStab with the unpreconditioned solver as fallback.

    The preconditioned solve (y_0 = 0, x = M y) runs with stall detection; if it ends in
    BREAKDOWN, ERR_NONFINITE or a stall, the true residual judges between x_0 = 0 and
    x = M y, and unpreconditioned p-BiCGStab restarts from the better one with the
    iterations left.  ``iterations`` counts both runs; ``fell_back`` is 1 after a restart.
    """
    spmv = spmv or _spmv
    dot = dot or default_dot(A.n)
    r1 = pbicgstab(A, b, tol=tol, max_iter=max_iter, M=M, dot=dot, spmv=spmv, stall_window=stall_window)
    if r1.status not in (BREAKDOWN, ERR_NONFINITE, STALLED):
        return r1
    xs = r1.x if (math.isfinite(r1.true_relres) and r1.true_relres < 1.0) else np.zeros(A.n)
    r2 = pbicgstab(A, b, x0=xs, tol=tol, max_iter=max(max_iter - r1.iterations, 0), dot=dot, spmv=spmv)
    r2.iterations += r1.iterations
    r2.fell_back = 1
    return r2


def ir_solve(A, b, tol=1e-10, inner_tol=0.1, max_iter=20000, max_outer=60, dot=None, spmv=None,
             stall=100, max_fp64=10000, x0=None, max_bad=1) -> Result:
    """FP64 iterative refinement around an FP32 p-BiCGStab with reliable updates.

    FP32 part: Algorithm 2 with FP32 matrix values, vectors and scalars, the
    compensated row-sequential FP32 SpMV (``oracle.spmv.spmv_f32``) and the plain
    sequential FP32 dot (``dot_f32_seq``); it accumulates a correction d (x0 = 0) to the FP64 iterate.
    FP64 part, a "reliable update" each time the FP32 iterations stop: x = x + nu d,
    r = b - A x (row-sequential FP64 SpMV), nu' = sqrt(exdot(r, r)); converged when
    nu' / ||b|| <= tol.  Otherwise the FP32 state is rebuilt from r / nu' and the same
    Krylov process continues: p is rescaled by fp32(nu / nu'), and w = A r, t = A w,
    s = A p, z = A s, v = A z are recomputed in FP32 (the replacement of the paper's
    residual-replacement variant), rho = (r_hat, r) and
    alpha = rho / ((r_hat, w) + beta (r_hat, s) - (beta omega)(r_hat, z)) follow with the
    kept beta and omega.  The FP32 iterations stop after an iteration whose recursive
    residual sqrt((r, r)) (relative to the last update) is <= inner_tol, or
    <= fp32(tol ||b|| / nu) (the solve looks converged), or on breakdown, a non-finite
    scalar, (y, y) = 0 (d = d + alpha p first), no new minimum for ``stall``
    iterations, or when the total reaches max_iter.  After a breakdown, stall or
    (y, y) = 0 the process restarts instead (r_hat = r, p = r, s = w, z = t).  An update
    that does not lower nu below the best so far means the FP32 process has reached
    the accuracy its operator allows (about u32 cond(A) relative): after ``max_bad``
    such updates (default 1) -- or ``max_outer`` updates, or max_iter FP32 iterations
    -- the solve finishes in FP64 p-BiCGStab from the best iterate with residual
    replacement every 50 iterations (a restart from a non-smooth residual attains less
    accuracy than the solve from b), ``fell_back`` = 1.
    (With max_bad > 1, x returns to the best iterate and the FP32 process restarts.)
    ``iterations`` counts FP32 iterations (plus the FP64 finish); ``outer_iterations``
    counts reliable updates.
    """
    from synthgen import CSR
    f = np.float32
    spmv = spmv or _spmv
    dot32 = dot_f32_seq
    n = A.n
    dot = dot or default_dot(n)
    b = np.asarray(b, dtype=np.float64)
    A32 = CSR(A.n, A.row_ptr, A.col_idx, A.val.astype(f))
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    normb = math.sqrt(dot(b, b))
    if normb == 0.0:
        return Result(np.zeros(n), OK, 0, 0.0, 0.0)
    if not math.isfinite(normb):
        return Result(x, ERR_NONFINITE, 0, math.nan, math.nan)
    delta = f(inner_tol)

    def residual(xv):
        r64 = b - spmv(A, xv)
        return r64, math.sqrt(dot(r64, r64))

    def finish(xs, its, outer):
        fin = pbicgstab(A, b, x0=xs, tol=tol, max_iter=max_fp64, dot=dot, spmv=spmv, rr_period=50)
        return Result(fin.x, fin.status, its + fin.iterations, fin.true_relres, fin.rec_relres,
                      fin.true_checks, outer_iterations=outer, fell_back=1)

    r64, nu = residual(x)
    if not math.isfinite(nu):
        return Result(x, ERR_NONFINITE, 0, math.nan, math.nan)
    if nu / normb <= tol:
        return Result(x, OK, 0, nu / normb, nu / normb)
    x_best, nu_best, bad, outer, its = x, nu, 0, 0, 0
    restart = True
    sigma = f(1.0)
    p = s = z = v = None
    alpha = beta = omega = rho = f(0.0)
    rec = f(1.0)
    while True:
        # rebuild the FP32 state from r / nu
        lim = f(tol * normb / nu)
        r = (r64 / nu).astype(f)
        w = _spmv_f32(A32, r)
        t = _spmv_f32(A32, w)
        if not restart:
            p = p * sigma
            s = _spmv_f32(A32, p)
            z = _spmv_f32(A32, s)
            v = _spmv_f32(A32, z)
            rho = dot32(rhat, r)
            rw = dot32(rhat, w)
            rs = dot32(rhat, s)
            rz = dot32(rhat, z)
            den = f(f(rw + f(beta * rs)) - f(f(beta * omega) * rz))
            if rho == 0 or den == 0 or not np.isfinite(den):
                restart = True
            else:
                alpha = f(rho / den)
        if restart:
            rhat = r.copy()
            rho = dot32(rhat, r)
            rw = dot32(rhat, w)
            if rw == 0 or not np.isfinite(rw):
                return finish(x_best, its, outer)
            alpha = f(rho / rw)
            beta = omega = f(0.0)
        first = restart
        best, it_best = math.inf, its
        d = np.zeros(n, dtype=f)
        reason = 0
        # FP32 iterations until a stop reason
        while not reason:
            if first:
                p, s, z = r.copy(), w.copy(), t.copy()
                first = False
            else:
                p = r + beta * (p - omega * s)
                s = w + beta * (s - omega * z)
                z = t + beta * (z - omega * v)
            q = r - alpha * s
            yv = w - alpha * z
            qy = dot32(q, yv)
            yy = dot32(yv, yv)
            rs = dot32(rhat, s)
            rz = dot32(rhat, z)
            v = _spmv_f32(A32, z)
            if yy == 0 or not np.isfinite(yy):
                if yy == 0:
                    d = d + alpha * p
                    its += 1
                    reason = _RU_YYZERO
                else:
                    reason = _RU_NONFINITE
                break
            om = f(qy / yy)
            if om == 0 or not np.isfinite(om):
                reason = _RU_BREAKDOWN
                break
            omega = om
            d = (d + alpha * p) + omega * q
            r = q - omega * yv
            w = yv - omega * (t - alpha * v)
            t = _spmv_f32(A32, w)
            rho_new = dot32(rhat, r)
            rw = dot32(rhat, w)
            rr = dot32(r, r)
            its += 1
            rec = f(np.sqrt(rr))
            bn = f(f(f(alpha / omega) * rho_new) / rho)
            den = f(f(rw + f(bn * rs)) - f(f(bn * omega) * rz))
            if rho_new == 0 or den == 0 or not np.isfinite(den):
                reason |= _RU_BREAKDOWN
            else:
                beta, alpha, rho = bn, f(rho_new / den), rho_new
            if rec <= lim:
                reason |= _RU_CONVERGED
            if rec <= delta:
                reason |= _RU_CHECK
            if rec < best:
                best, it_best = rec, its
            elif stall > 0 and its - it_best >= stall:
                reason |= _RU_STALL
            if its >= max_iter:
                reason |= _RU_MAXIT
        # reliable update
        x = x + nu * d.astype(np.float64)
        r64, nu_new = residual(x)
        outer += 1
        if not math.isfinite(nu_new):
            return finish(x_best, its, outer)
        if nu_new / normb <= tol:
            return Result(x, OK, its, nu_new / normb, float(rec) * nu / normb, outer_iterations=outer)
        restart = bool(reason & _RU_RESTART)
        if nu_new < nu_best:
            x_best, nu_best, bad = x, nu_new, 0
        else:
            bad += 1
            restart = True
            x = x_best
            r64, nu_new = residual(x)
        if bad >= max_bad or outer >= max_outer or (reason & _RU_MAXIT):
            return finish(x_best, its, outer)
        sigma = f(nu / nu_new)
        nu = nu_new




def pbicgstab_fp32_matrix(A, b, tol=1e-10, max_iter=10000, rr_period=50, dot=None, history=False) -> Result:
    """FP64 p-BiCGStab whose iterations apply A's values rounded to FP32 (vectors, the
    accumulation of every row and all scalars stay FP64; inner products exact), with
    residual replacement against the FP64 A every rr_period iterations: r = b - A x with
    the FP64 values, then w, t, s, z, v recomputed with the FP32 ones.  ||b||, r_0 and the
    true residual that decides convergence use the FP64 A.  (The build's precision form:
    half the value bytes per SpMV, FP64 Krylov vectors.)"""
    from synthgen import CSR
    A32 = CSR(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32).astype(np.float64))
    dot = dot or default_dot(A.n)
    return pbicgstab(A32, b, tol=tol, max_iter=max_iter, dot=dot, rr_period=rr_period,
                     resid=lambda _A, b_, x_: b_ - _spmv(A, x_), record=0)
