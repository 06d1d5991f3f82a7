"""CSR sparse matrix-vector product, sequential row sums -- oracle.

Algorithms 1 and 2 of the paper apply A to a vector (A p_i, A q_i, A z_i, A w_i)
without fixing a storage format or a summation order.  Reading used here: CSR,
and row i is summed left to right in storage order,

    s = 0;  for k in row i:  s = s + (a_k * x[col_k])

with the multiply and the add rounded separately (no fused multiply-add).
The GPU sums rows in a different (tree) order, so SpMV results agree only up to
the classical bound |y - y_exact| <= gamma_len * sum_k |a_k x_col_k|.
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
    """Row-sequential SpMV in float32 arithmetic (values, vector and accumulator)."""
    rp = A32.row_ptr.astype(np.int64)
    lens = np.diff(rp)
    y = np.zeros(A32.n, dtype=np.float32)
    kmax = int(lens.max()) if lens.size else 0
    for k in range(kmax):
        rows = np.nonzero(lens > k)[0]
        idx = rp[rows] + k
        y[rows] = y[rows] + A32.val[idx] * x32[A32.col_idx[idx]]
    return y
