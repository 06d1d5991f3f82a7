"""BiCGStab (Algorithm 1) and p-BiCGStab (Algorithm 2) over the rationals -- oracle.

Exact arithmetic (``fractions.Fraction``) for tiny systems.  The paper states that
the two algorithms are mathematically equivalent (Section 2, the paragraph after
the algorithms); in exact arithmetic their iterates must coincide, and without
breakdown BiCGStab terminates with r = 0 in at most n iterations.  These
properties pin the FP64 oracle's recurrences (a dropped term, a wrong sign or a
misplaced index breaks the equality).  Same readings of Algorithm 2 as
``oracle.solvers``.
"""
from __future__ import annotations

from fractions import Fraction as F


def _dense(A):
    n = A.n
    M = [[F(0)] * n for _ in range(n)]
    for i in range(n):
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            M[i][int(A.col_idx[k])] = F(float(A.val[k]))
    return M


def _mv(M, x):
    return [sum((a * b for a, b in zip(row, x)), F(0)) for row in M]


def _dot(a, b):
    return sum((u * v for u, v in zip(a, b)), F(0))


def _axpy(a, x, y):  # y + a x
    return [v + a * u for u, v in zip(x, y)]


def bicgstab_q(A, b, iters):
    """Iterates x_1..x_iters of Algorithm 1 in exact arithmetic (stops early if r = 0)."""
    M = _dense(A)
    bq = [F(float(v)) for v in b]
    x = [F(0)] * A.n
    r = list(bq)
    rhat = list(r)
    p = list(r)
    rho = _dot(rhat, r)
    xs = []
    for _ in range(iters):
        s = _mv(M, p)
        alpha = rho / _dot(rhat, s)
        q = _axpy(-alpha, s, r)
        y = _mv(M, q)
        yy = _dot(y, y)
        if yy == 0:
            x = _axpy(alpha, p, x)
            xs.append(x)
            break
        omega = _dot(q, y) / yy
        x = _axpy(omega, q, _axpy(alpha, p, x))
        r = _axpy(-omega, y, q)
        xs.append(x)
        if all(v == 0 for v in r):
            break
        rho_new = _dot(rhat, r)
        beta = (alpha / omega) * rho_new / rho
        p = _axpy(beta, _axpy(-omega, s, p), r)
        rho = rho_new
    return xs


def pbicgstab_q(A, b, iters):
    """Iterates x_1..x_iters of Algorithm 2 in exact arithmetic."""
    M = _dense(A)
    bq = [F(float(v)) for v in b]
    x = [F(0)] * A.n
    r = list(bq)
    rhat = list(r)
    w = _mv(M, r)
    t = _mv(M, w)
    rho = _dot(rhat, r)
    alpha = rho / _dot(rhat, w)
    beta = omega = F(0)
    p = s = z = v = None
    xs = []
    for i in range(iters):
        if i == 0:
            p, s, z = list(r), list(w), list(t)
        else:
            p = _axpy(beta, _axpy(-omega, s, p), r)
            s = _axpy(beta, _axpy(-omega, z, s), w)
            z = _axpy(beta, _axpy(-omega, v, z), t)
        q = _axpy(-alpha, s, r)
        y = _axpy(-alpha, z, w)
        v = _mv(M, z)
        yy = _dot(y, y)
        if yy == 0:
            x = _axpy(alpha, p, x)
            xs.append(x)
            break
        omega = _dot(q, y) / yy
        x = _axpy(omega, q, _axpy(alpha, p, x))
        r = _axpy(-omega, y, q)
        w = _axpy(-omega, _axpy(-alpha, v, t), y)
        t = _mv(M, w)
        xs.append(x)
        if all(u == 0 for u in r):
            break
        rho_new = _dot(rhat, r)
        beta = (alpha / omega) * rho_new / rho
        alpha = rho_new / (_dot(rhat, w) + beta * _dot(rhat, s) - beta * omega * _dot(rhat, z))
        rho = rho_new
    return xs
