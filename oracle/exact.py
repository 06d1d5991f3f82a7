"""Exact dot product rounded once to FP64 -- oracle tier 1 (pure Python integers).

Paper, Section 2 (ExBLAS paragraph): the reproducible p-BiCGStab accumulates
every inner product with a long accumulator plus floating-point expansions so
that the result does not depend on partitioning, operation order, thread
scheduling or reduction tree.  The plain definition of such a result is

    exdot(x, y) = RN_even( sum_i x_i * y_i )      (the sum taken exactly)

which is what this module computes.  Readings where the paper is silent:

* rounding is round-to-nearest, ties-to-even;
* an exact zero sum returns +0.0, n = 0 returns +0.0; a non-zero sum that
  underflows keeps its sign (-0.0 for tiny negative sums);
* |exact| >= 2^1024 - 2^970 rounds to +-inf;
* non-finite inputs: any NaN, any inf*0, or both +inf and -inf products give the
  canonical quiet NaN; otherwise any +-inf product gives that infinity.
  Products of finite inputs are always exact, even when they exceed DBL_MAX or
  fall below the subnormal range.

Every product of finite doubles is an integer multiple of 2^-2148, so the exact
sum is S * 2^-2148 for a Python integer S; CPython's int / int true division is
correctly rounded (ties to even), which performs the single rounding.
"""
from __future__ import annotations

import math
from typing import Iterable

SCALE = 2148  # -(exponent of the lowest bit of any product): 2 * 1074


def split(d: float) -> tuple[int, int]:
    """d = m * 2**e exactly with integer m (signed) -- d finite."""
    num, den = d.as_integer_ratio()
    return num, -(den.bit_length() - 1)


def scaled_product(a: float, b: float) -> int:
    """a*b*2^2148 as an exact integer (a, b finite)."""
    ma, ea = split(a)
    mb, eb = split(b)
    sh = ea + eb + SCALE
    assert sh >= 0
    return (ma * mb) << sh


def round_scaled(S: int) -> float:
    """RN_even(S * 2^-2148) with the zero / overflow readings above."""
    if S == 0:
        return 0.0
    try:
        return S / (1 << SCALE)
    except OverflowError:
        return math.inf if S > 0 else -math.inf


def _nonfinite(pairs: Iterable[tuple[float, float]]):
    nan = pinf = ninf = False
    for a, b in pairs:
        if math.isnan(a) or math.isnan(b):
            nan = True
        elif math.isinf(a) or math.isinf(b):
            if a == 0.0 or b == 0.0:
                nan = True
            elif (a > 0) == (b > 0):
                pinf = True
            else:
                ninf = True
    return nan, pinf, ninf


def exact_sum_scaled(x, y) -> int:
    """S with sum_i x_i y_i = S * 2^-2148 (all inputs finite)."""
    S = 0
    for a, b in zip(x, y):
        if a == 0.0 or b == 0.0:
            continue
        S += scaled_product(float(a), float(b))
    return S


def exact_dot(x, y) -> float:
    """RN_even of the exact dot product of two equal-length sequences of doubles."""
    xs = [float(v) for v in x]
    ys = [float(v) for v in y]
    if len(xs) != len(ys):
        raise ValueError("length mismatch")
    if not all(math.isfinite(v) for v in xs) or not all(math.isfinite(v) for v in ys):
        nan, pinf, ninf = _nonfinite(zip(xs, ys))
        if nan or (pinf and ninf):
            return math.nan
        if pinf:
            return math.inf
        if ninf:
            return -math.inf
    return round_scaled(exact_sum_scaled(xs, ys))


def exact_sum(x) -> float:
    """RN_even of the exact sum of a sequence of doubles (dot with ones)."""
    return exact_dot(x, [1.0] * len(x))
