"""GPU exact dot product vs the oracle: bit-exact, and bit-identical across launch shapes.

The oracle's exact dot (paper Section 2, ExBLAS: accumulated exactly, rounded once)
is RN_even(sum x_i y_i); the GPU result must have the same bits for every input
family -- random, wide exponent ranges, tiny products below the subnormal range,
products beyond DBL_MAX, heavy cancellation, non-finite inputs -- and for every grid,
block size and expansion length.
"""
import json
import os

import numpy as np
import pytest

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier, exact
from tests.gpu_util import same_bits, to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "exdot_cases.jsonl")


def gpu_dot(x, y, **cfg):
    tx, ty = to_dev(np.asarray(x, dtype=np.float64)), to_dev(np.asarray(y, dtype=np.float64))
    if cfg:
        return pk.exdot_config(tx, ty, cfg["grid"], cfg["block"], cfg["k"]).item()
    return pk.exdot(tx, ty).item()


def families(n, seed):
    rng = np.random.default_rng(seed)
    yield "uniform", rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    yield "normal_scaled", rng.standard_normal(n) * 1e-3, rng.standard_normal(n) * 1e5
    yield "wide", g.wide_exponent_vec(n, seed, -500, 500), g.wide_exponent_vec(n, seed + 1, -500, 500)
    yield "tiny", g.wide_exponent_vec(n, seed, -1074, -480), g.wide_exponent_vec(n, seed + 2, -700, -400)
    yield "huge", g.wide_exponent_vec(n, seed, 400, 1023), g.wide_exponent_vec(n, seed + 3, 500, 1023)
    yield "full_range", g.wide_exponent_vec(n, seed, -1074, 1023), g.wide_exponent_vec(n, seed + 4, -1074, 1023)
    a = rng.standard_normal(n // 2) * 2.0 ** rng.integers(-60, 60, n // 2)
    x = np.concatenate([a, a, rng.standard_normal(n - 2 * (n // 2))])
    y = np.concatenate([np.ones(n // 2), -np.ones(n // 2), rng.standard_normal(n - 2 * (n // 2)) * 1e-30])
    yield "cancel", x, y
    i = np.arange(1, n + 1, dtype=np.float64)
    yield "closed_form", i, i


def _golden():
    for line in open(GOLD):
        c = json.loads(line)
        yield ([float.fromhex(v) for v in c["x"]], [float.fromhex(v) for v in c["y"]],
               float.fromhex(c["expected"]), c["why"])


@pytest.mark.parametrize("case", list(_golden()), ids=lambda c: c[3][:40])
def test_golden(case):
    x, y, e, why = case
    if len(x) == 0:
        x, y = [0.0], [0.0]  # zero-length handled separately
    assert same_bits(gpu_dot(x, y), e), why


def test_empty():
    import torch
    t = torch.empty(0, dtype=torch.float64, device="cuda:0")
    assert same_bits(pk.exdot(t, t).item(), 0.0)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 4097, 65536 + 17, 300001])
def test_families_vs_oracle(n):
    for name, x, y in families(n, n):
        ref = ctier.exact_dot(x, y)
        got = gpu_dot(x, y)
        assert same_bits(got, ref), (name, n, got, ref)


def test_tier1_crosscheck_small():
    for name, x, y in families(3000, 5):
        assert same_bits(gpu_dot(x, y), exact.exact_dot(x.tolist(), y.tolist())), name


def test_nonfinite_inputs():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000)
    y = rng.standard_normal(10000)
    for pos, val, other, expect in [(17, np.nan, 1.0, "nan"), (9000, np.inf, 0.0, "nan"),
                                    (5, np.inf, 2.0, "inf"), (6, -np.inf, 3.0, "-inf")]:
        xx, yy = x.copy(), y.copy()
        xx[pos] = val
        yy[pos] = other
        got = gpu_dot(xx, yy)
        assert same_bits(got, float(expect)) and same_bits(got, ctier.exact_dot(xx, yy))
    xx = x.copy()
    xx[3], xx[9999] = np.inf, -np.inf
    yy = np.ones_like(x)
    assert np.isnan(gpu_dot(xx, yy))


@pytest.mark.parametrize("fam", ["uniform", "wide", "tiny", "full_range", "cancel"])
def test_launch_shape_invariance(fam):
    n = 200003
    x, y = {k: (a, b) for k, a, b in families(n, 11)}[fam]
    ref = ctier.exact_dot(x, y)
    for grid in (1, 3, 64, 1024):
        for block in (64, 256, 1024):
            for k in (2, 3, 4, 6, 8):
                if grid == 1024 and block == 1024 and k > 4:
                    continue
                got = gpu_dot(x, y, grid=grid, block=block, k=k)
                assert same_bits(got, ref), (fam, grid, block, k, got, ref)


def test_full_size_2pow24():
    """Workload size of the largest vectors of the 128^3 and 256^3 problems."""
    n = 1 << 24
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, n)
    y = rng.standard_normal(n)
    assert same_bits(gpu_dot(x, y), ctier.exact_dot(x, y))
    x[::7] *= 1e-200
    assert same_bits(gpu_dot(x, y), ctier.exact_dot(x, y))


def test_run_to_run_bitwise():
    x, y = g.wide_exponent_vec(100000, 1, -300, 300), g.wide_exponent_vec(100000, 2, -300, 300)
    vals = {np.float64(gpu_dot(x, y)).view(np.uint64) for _ in range(5)}
    assert len(vals) == 1
