"""CSR sparse matrix-vector product, sequential row sums -- oracle.

Algorithms 1 and 2 of the paper apply A to a vector (A p_i, A q_i, A z_i, A w_i)
without fixing a storage format or a summation order.  Reading used here: CSR,
and row i is summed left to right in storage order,

    s = 0;  for k in row i:  s = s + (a_k * x[col_k])

with the multiply and the add rounded separately (no fused multiply-add).
The GPU's row-sequential kernels use the same order and agree bit for bit; its
vector and wavefront kernels sum rows as trees, which agree up to the classical bound
|y - y_exact| <= gamma_len * sum_k |a_k x_col_k|.
"""
from __future__ import annotations

import numpy as np


def spmv(A, x: np.ndarray) -> np.ndarray:
    """y = A x, row-sequential, vectorised over rows slot by slot."""
    rp = A.row_ptr.astype(np.int64)
    lens = np.diff(rp)
    y = np.zeros(A.n, dtype=np.float64)
    if A.n == 0:
        return y
    kmax = int(lens.max()) if lens.size else 0
    x = np.asarray(x, dtype=np.float64)
    for k in range(kmax):
        rows = np.nonzero(lens > k)[0]
        idx = rp[rows] + k
        y[rows] = y[rows] + A.val[idx] * x[A.col_idx[idx]]
    return y


def spmv_loops(A, x) -> list:
    """The same sum written as plain Python loops (tiny inputs only)."""
    out = []
    for i in range(A.n):
        s = 0.0
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            s = s + float(A.val[k]) * float(x[int(A.col_idx[k])])
        out.append(s)
    return out


def spmv_abs(A, x: np.ndarray) -> np.ndarray:
    """sum_k |a_k x_col_k| per row (for error bounds)."""
    return spmv(type(A)(A.n, A.row_ptr, A.col_idx, np.abs(A.val)), np.abs(x))


def spmv_f32(A32, x32: np.ndarray) -> np.ndarray:
    """Row-sequential SpMV in float32 with compensated accumulation: algorithm Dot2 of
    Ogita, Rump and Oishi ("Accurate sum and dot product", SIAM J. Sci. Comput. 2005)
    applied to every row in storage order.  Starting from s = c = 0, for each entry

        p = fl(a x),  e = a x - p                      (TwoProduct: e is exact)
        s' = fl(s + p),  b = fl(s' - s),
        err = fl(fl(s - fl(s' - b)) + fl(p - b))       (TwoSum, Knuth: s + p = s' + err)
        c = fl(c + fl(err + e)),  s = s'

    and the row's result is fl(s + c).  Every operation is float32; the product error
    e is taken from the exact float64 product a x (a 48-bit significand) minus p, which
    is the same value a fused multiply-add fma(a, x, -p) returns.  The result is as
    accurate as a sum in twice the working precision, rounded once.
    """
    f = np.float32
    rp = A32.row_ptr.astype(np.int64)
    lens = np.diff(rp)
    s = np.zeros(A32.n, dtype=f)
    c = np.zeros(A32.n, dtype=f)
    kmax = int(lens.max()) if lens.size else 0
    x32 = np.asarray(x32, dtype=f)
    for k in range(kmax):
        rows = np.nonzero(lens > k)[0]
        idx = rp[rows] + k
        a = A32.val[idx].astype(f)
        xv = x32[A32.col_idx[idx]]
        ax = a.astype(np.float64) * xv.astype(np.float64)
        pr = ax.astype(f)
        e = (ax - pr.astype(np.float64)).astype(f)
        so = s[rows]
        sn = so + pr
        bb = sn - so
        err = (so - (sn - bb)) + (pr - bb)
        s[rows] = sn
        c[rows] = c[rows] + (err + e)
    return s + c


def spmv_f32_loops(A32, x32) -> list:
    """The same Dot2 row sums written as plain loops over numpy float32 scalars, with
    the product error from Python's exact rational arithmetic (tiny inputs only)."""
    from fractions import Fraction
    f = np.float32
    out = []
    for i in range(A32.n):
        s = f(0.0)
        c = f(0.0)
        for k in range(int(A32.row_ptr[i]), int(A32.row_ptr[i + 1])):
            a = f(A32.val[k])
            xv = f(x32[int(A32.col_idx[k])])
            p = a * xv
            e = f(float(Fraction(float(a)) * Fraction(float(xv)) - Fraction(float(p))))
            sn = s + p
            bb = sn - s
            err = (s - (sn - bb)) + (p - bb)
            s = sn
            c = c + (err + e)
        out.append(s + c)
    return out


# ---------------------------------------------------------------------------
# Exactly rounded rows (the ExBLAS idea of the paper's Section 2 applied to the rows of
# A x): every row's sum is formed exactly and rounded once to nearest-even, so the result
# depends on no summation order at all.
# ---------------------------------------------------------------------------
def _row_dot(a, b):
    from . import exact
    if len(a) <= 64:
        return exact.exact_dot(list(a), list(b))
    from . import ctier
    return ctier.exact_dot(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))


def spmv_exact(A, x, rows=None) -> np.ndarray:
    """y_i = RN(sum_k a_ik x_k), each row one exact dot product rounded once (rows: an
    optional subset; the returned vector then holds those rows only)."""
    x = np.asarray(x, dtype=np.float64)
    rp = A.row_ptr
    idx = range(A.n) if rows is None else rows
    out = []
    for i in idx:
        a, e = int(rp[i]), int(rp[i + 1])
        out.append(_row_dot(np.asarray(A.val[a:e], dtype=np.float64).tolist(), x[A.col_idx[a:e]].tolist()))
    return np.array(out, dtype=np.float64)


def resid_exact(A, b, x, rows=None) -> np.ndarray:
    """r_i = RN(b_i - sum_k a_ik x_k): the residual row as one exact sum, rounded once
    (b_i enters as the term b_i * 1)."""
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    rp = A.row_ptr
    idx = range(A.n) if rows is None else rows
    out = []
    for i in idx:
        a, e = int(rp[i]), int(rp[i + 1])
        vals = [float(b[i])] + (-np.asarray(A.val[a:e], dtype=np.float64)).tolist()
        xs = [1.0] + x[A.col_idx[a:e]].tolist()
        out.append(_row_dot(vals, xs))
    return np.array(out, dtype=np.float64)
