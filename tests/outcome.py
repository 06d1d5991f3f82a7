"""Outcome checks for solves whose iterates cannot match the oracle bit for bit (the
FP32 refinement and the ordinary-dot comparator: their plain dots are formed in the
library's fixed reduction tree, the oracle's in the sequential order of the definition).

Such a solve is judged by what it reaches:

* its true relative residual ||b - A x||_2 / ||b||_2, recomputed here from the returned x
  by the oracle (row-sequential FP64 SpMV, exact dots), must meet the tolerance;
* its distance from a reference solution is bounded by perturbation theory: with
  r = b - A x and r' = b - A x' (both formed exactly), x - x' = A^-1 (r' - r), so

      ||x - x'||_inf <= ||A^-1||_inf (||r||_inf + ||r'||_inf),

  where the computed residuals carry a rounding slack of gamma_(k+1) max_i(|b_i| +
  sum_j |a_ij x_j|) each (k the longest row; Higham's bound for a sequential sum).

||A^-1||_inf is bounded from above with a certificate that holds for every family here:

* strict row diagonal dominance (the random family): Varah's bound
  ||A^-1||_inf <= 1 / min_i (|a_ii| - sum_(j != i) |a_ij|);
* a Z-matrix (the upwind convection-diffusion stencils: off-diagonals <= 0) and a
  vector v > 0 with A v >= c > 0 componentwise: A is then a nonsingular M-matrix,
  A^-1 >= 0, A^-1 1 <= v / c, and ||A^-1||_inf = ||A^-1 1||_inf <= max(v) / c.  The
  candidate v may come from anywhere (a sparse LU here, or any solver); only the
  inequality, checked with the oracle's SpMV and its rounding bound, is trusted.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ctier
from oracle.spmv import spmv

U64 = 2.0 ** -53


def gamma(k: int) -> float:
    return k * U64 / (1.0 - k * U64)


def _abs_csr(A):
    import synthgen as g
    return g.CSR(A.n, A.row_ptr, A.col_idx, np.abs(A.val))


def max_row_len(A) -> int:
    return int(np.diff(A.row_ptr.astype(np.int64)).max(initial=0))


def residual(A, b, x):
    """r = b - A x by the oracle's row-sequential SpMV, and the bound on its rounding
    error in the inf-norm."""
    b = np.asarray(b, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    r = b - spmv(A, x)
    slack = gamma(max_row_len(A) + 1) * float(np.max(np.abs(b) + spmv(_abs_csr(A), np.abs(x)), initial=0.0))
    return r, slack


def true_relres(A, b, x) -> float:
    """The oracle's true relative residual sqrt(exdot(r, r)) / sqrt(exdot(b, b))."""
    r = np.asarray(b, dtype=np.float64) - spmv(A, np.asarray(x, dtype=np.float64))
    return math.sqrt(ctier.exact_dot(r, r)) / math.sqrt(ctier.exact_dot(b, b))


def _split(A):
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    diag = rows == A.col_idx
    return rows, diag


def inv_norm_inf_bound(A, v=None) -> float:
    """A certified upper bound on ||A^-1||_inf (see the module docstring).  For a
    Z-matrix without strict diagonal dominance, `v` is the candidate vector; None
    computes it with scipy's sparse LU (test-sized matrices only)."""
    rows, diag = _split(A)
    absval = np.abs(A.val)
    dvals = np.zeros(A.n)
    dvals[rows[diag]] = absval[diag]
    off = np.bincount(rows[~diag], weights=absval[~diag], minlength=A.n)
    margin = dvals - off
    if np.all(margin > 0):
        # margin is computed in FP64: allow for the rounding of the off-diagonal sums
        lo = margin - gamma(max_row_len(A)) * off
        if np.all(lo > 0):
            return 1.0 / float(lo.min())
    if np.any(A.val[~diag] > 0) or np.any(A.val[diag] <= 0):
        raise ValueError("no certificate: neither strictly diagonally dominant nor a Z-matrix")
    if v is None:
        import scipy.sparse as sp
        import scipy.sparse.linalg as spl
        S = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n)).tocsc()
        v = spl.splu(S).solve(np.ones(A.n))
    v = np.asarray(v, dtype=np.float64)
    if not np.all(v > 0):
        # shift an approximate candidate to positive values; the inequality below is
        # checked on the shifted vector itself, so nothing is assumed about the shift
        v = v - min(float(v.min()), 0.0) + 1e-9 * float(np.abs(v).max())
    if not np.all(v > 0):
        raise ValueError("candidate vector is not positive")
    Av = spmv(A, v)
    err = gamma(max_row_len(A)) * spmv(_abs_csr(A), v)
    c = float((Av - err).min())
    if not c > 0:
        raise ValueError("certificate failed: A v is not positive")
    return float(v.max()) / c


def solution_gap_bound(A, b, x, xref, inv_norm=None) -> float:
    """Upper bound on ||x - xref||_inf from the two residuals."""
    r, e = residual(A, b, x)
    r2, e2 = residual(A, b, xref)
    if inv_norm is None:
        inv_norm = inv_norm_inf_bound(A)
    return inv_norm * (float(np.abs(r).max()) + e + float(np.abs(r2).max()) + e2)
