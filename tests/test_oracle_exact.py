"""Pins of the oracle's exact dot product (rounded once; paper Section 2, ExBLAS).

Each pin is something other than the oracle itself: values fixed by hand from
the IEEE 754 round-to-nearest-even definition (tests/golden/exdot_cases.jsonl),
``math.fsum`` (Shewchuk's correctly rounded summation, a library routine) on
inputs whose products are exact or split exactly by Dekker's TwoProduct, a
brute-force Fraction sum rounded by an independent integer RNE, closed forms,
and agreement of the two independently written tiers (Python ints, C limbs).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ctier, exact
import synthgen as g

GOLD = os.path.join(os.path.dirname(__file__), "golden", "exdot_cases.jsonl")


def _same(a, b):
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b and math.copysign(1.0, a) == math.copysign(1.0, b)


def _golden():
    out = []
    for line in open(GOLD):
        c = json.loads(line)
        out.append(([float.fromhex(v) for v in c["x"]], [float.fromhex(v) for v in c["y"]],
                     float.fromhex(c["expected"]), c["why"]))
    return out


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[3][:40])
def test_golden_tier1(case):
    x, y, e, _ = case
    assert _same(exact.exact_dot(x, y), e)


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[3][:40])
def test_golden_tier2(case):
    x, y, e, _ = case
    assert _same(ctier.exact_dot(np.array(x), np.array(y)), e)


def rne_fraction(q: Fraction) -> float:
    """Independent round-to-nearest-even of a rational to binary64 (integer arithmetic)."""
    if q == 0:
        return 0.0
    neg = q < 0
    q = -q if neg else q
    N, D = q.numerator, q.denominator
    # leading exponent L with 2^L <= q < 2^(L+1)
    L = N.bit_length() - D.bit_length()
    if (N << max(0, -L)) < (D << max(0, L)):
        L -= 1
    e = max(L - 52, -1074)            # exponent of the last place
    # m = floor(q / 2^e), remainder test for round bit
    num = N << max(0, -e)
    den = D << max(0, e)
    m, rem = divmod(num, den)
    if 2 * rem > den or (2 * rem == den and (m & 1)):
        m += 1
    if m == 1 << 53:
        m >>= 1
        e += 1
    if e + 52 > 1023 and m >= 1 << 52:
        r = math.inf
    else:
        r = math.ldexp(m, e)
    return -r if neg else r


def brute(x, y):
    return rne_fraction(sum((Fraction(a) * Fraction(b) for a, b in zip(x, y)), Fraction(0)))


def test_independent_rounding_on_goldens():
    for x, y, e, why in _golden():
        if all(math.isfinite(v) for v in x + y):
            r = brute(x, y)
            if r == 0.0 and e == 0.0:
                continue  # sign of an exact zero is a convention, checked in the goldens
            assert _same(r, e), why


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_fraction_random(seed):
    rng = np.random.default_rng(seed)
    n = 60
    fam = seed % 3
    if fam == 0:
        x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    elif fam == 1:
        x, y = g.wide_exponent_vec(n, seed, -600, 500), g.wide_exponent_vec(n, seed + 100, -600, 500)
    else:  # heavy cancellation: pairs that cancel exactly plus small residue
        a = rng.uniform(-1, 1, n // 2) * 2.0 ** rng.integers(-40, 40, n // 2)
        x = np.concatenate([a, a])
        y = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
        y[3] = 1.0 + 2.0 ** -40
    r1 = exact.exact_dot(x.tolist(), y.tolist())
    assert _same(r1, brute(x.tolist(), y.tolist()))


def two_prod_dekker(a, b):
    """Dekker's TwoProduct with Veltkamp splitting (exact without over/underflow)."""
    def split(v):
        c = 134217729.0 * v
        hi = c - (c - v)
        return hi, v - hi
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


@pytest.mark.parametrize("seed", range(8))
def test_fsum_of_dekker_pairs(seed):
    rng = np.random.default_rng(100 + seed)
    n = 2000
    x = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-200, 200, n)
    y = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-200, 200, n)
    terms = []
    for a, b in zip(x.tolist(), y.tolist()):
        terms.extend(two_prod_dekker(a, b))
    ref = math.fsum(terms)
    assert _same(exact.exact_dot(x.tolist(), y.tolist()), ref)
    assert _same(ctier.exact_dot(x, y), ref)


@pytest.mark.parametrize("seed", range(4))
def test_fsum_sum_of_doubles(seed):
    """exdot(x, 1) is the correctly rounded sum, i.e. math.fsum(x)."""
    x = g.wide_exponent_vec(5000, seed, -1070, 1000)
    ref = math.fsum(x.tolist())
    assert _same(exact.exact_sum(x.tolist()), ref)
    assert _same(ctier.exact_dot(x, np.ones_like(x)), ref)


def test_closed_forms():
    for n in (1, 7, 1000, 123457):
        i = np.arange(1, n + 1, dtype=np.float64)
        assert ctier.exact_dot(i, np.ones(n)) == n * (n + 1) / 2
        s2 = n * (n + 1) * (2 * n + 1) // 6
        assert ctier.exact_dot(i, i) == float(s2)  # int -> float conversion is RNE
    n = 5000
    i = np.arange(1, n + 1, dtype=np.float64)
    assert exact.exact_dot(i.tolist(), i.tolist()) == float(n * (n + 1) * (2 * n + 1) // 6)


def test_order_and_partition_invariance():
    rng = np.random.default_rng(7)
    x = g.wide_exponent_vec(3000, 1, -500, 500)
    y = rng.uniform(-1, 1, 3000)
    r = ctier.exact_dot(x, y)
    perm = rng.permutation(3000)
    assert _same(ctier.exact_dot(x[perm], y[perm]), r)
    # split into chunks, accumulate exactly, same result
    parts = [exact.exact_sum_scaled(x[k:k + 700].tolist(), y[k:k + 700].tolist())
             for k in range(0, 3000, 700)]
    assert _same(exact.round_scaled(sum(parts)), r)


@pytest.mark.parametrize("seed", range(5))
def test_tier1_equals_tier2_random(seed):
    rng = np.random.default_rng(seed)
    for fam in range(4):
        n = int(rng.integers(0, 3000))
        if fam == 0:
            x, y = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        elif fam == 1:
            x, y = g.wide_exponent_vec(n, seed, -1074, 1023), g.wide_exponent_vec(n, seed + 9, -1074, 1023)
        elif fam == 2:
            x, y = g.wide_exponent_vec(n, seed, -1074, -400), g.wide_exponent_vec(n, seed + 9, -700, 0)
        else:
            x = rng.standard_normal(n)
            y = np.concatenate([x[: n // 2], -x[: n // 2], rng.standard_normal(n - 2 * (n // 2))]) if n else x
            x = np.concatenate([x[: n // 2], x[: n // 2], rng.standard_normal(n - 2 * (n // 2))]) if n else x
        assert _same(exact.exact_dot(x.tolist(), y.tolist()), ctier.exact_dot(x, y))


def _round_cases():
    rng = np.random.default_rng(11)
    S = []
    one = 1 << exact.SCALE
    for _ in range(300):
        bits = int(rng.integers(1, 4300))
        v = int(rng.integers(1, 2 ** 62)) << max(0, bits - 62)
        v |= int(rng.integers(0, 2 ** 30))
        S.append(v if rng.random() < 0.5 else -v)
    for k in range(-1074, 1024, 37):  # ties and near-ties at many exponents
        base = (1 << 52 | 12345) << (k + exact.SCALE - 52) if k >= -1022 else 3 << (1074 - 1074)
        ulp = 1 << max(0, k - 52 + exact.SCALE) if k >= -1022 else 1 << (exact.SCALE - 1074)
        for d in (ulp // 2, ulp // 2 - 1, ulp // 2 + 1, 0):
            S.append(base + d)
            S.append(-(base + d))
    S += [one, -one, 1, -1, (1 << 1074) - 1]
    return S


def test_rounding_tiers_agree():
    """CPython's int/int division and the C limb rounding are independent codes."""
    for s in _round_cases():
        assert _same(exact.round_scaled(s), ctier.round_limbs(s)), s
