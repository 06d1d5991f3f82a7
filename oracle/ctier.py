"""ctypes binding of the C tier of the oracle (oracle/c/oracle.c) -- test infrastructure.

``build()`` compiles ``oracle/c/liboracle.so`` with gcc (-O2 -ffp-contract=off
-fopenmp); the module loads an existing build and builds only when none exists.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "oracle.c")
LIB = os.path.join(_HERE, "c", "liboracle.so")
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fPIC", "-shared", "-std=gnu11", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("true_checks", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("true_relres", ctypes.c_double), ("rec_relres", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.ora_exact_dot.restype = ctypes.c_double
        L.ora_exact_dot.argtypes = [P, P, ctypes.c_int64]
        L.ora_round_limbs.restype = ctypes.c_double
        L.ora_round_limbs.argtypes = [P]
        L.ora_spmv.restype = None
        L.ora_spmv.argtypes = [ctypes.c_int32, P, P, P, P, P]
        for f in (L.ora_pbicgstab, L.ora_bicgstab):
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                          ctypes.POINTER(Info), P]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def exact_dot(x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if x.shape != y.shape:
        raise ValueError("length mismatch")
    return float(lib().ora_exact_dot(_p(x), _p(y), x.size))


def round_limbs(S: int) -> float:
    """Round S * 2^-2148 (S a Python int, |S| < 2^4351) through the C rounding."""
    mask = (1 << 64) - 1
    u = S & ((1 << (68 * 64)) - 1)  # two's complement in 68 limbs
    limbs = np.array([(u >> (64 * k)) & mask for k in range(68)], dtype=np.uint64)
    return float(lib().ora_round_limbs(_p(limbs)))


def spmv(A, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n)
    lib().ora_spmv(A.n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), _p(x), _p(y))
    return y


def _solve(fn, A, b, x0, tol, max_iter, history):
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    info = Info()
    hist = np.full(max(max_iter, 1), np.nan) if history else None
    fn(A.n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), _p(b), _p(x), tol, max_iter,
       ctypes.byref(info), _p(hist) if history else None)
    out = dict(x=x, status=info.status, iterations=info.iterations, true_checks=info.true_checks,
               true_relres=info.true_relres, rec_relres=info.rec_relres)
    if history:
        out["history"] = hist[:info.iterations]
    return out


def pbicgstab(A, b, x0=None, tol=1e-10, max_iter=10000, history=False) -> dict:
    return _solve(lib().ora_pbicgstab, A, b, x0, tol, max_iter, history)


def bicgstab(A, b, x0=None, tol=1e-10, max_iter=10000, history=False) -> dict:
    return _solve(lib().ora_bicgstab, A, b, x0, tol, max_iter, history)


def set_threads(nt: int) -> None:
    lib().ora_set_threads(nt)


def num_threads() -> int:
    return int(lib().ora_num_threads())
