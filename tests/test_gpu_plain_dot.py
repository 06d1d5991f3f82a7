"""The library's plain (not exact) dot products -- the FP32 solver's inner products and
the ordinary-dot comparator's FP64 ones -- against the oracle's exact dot.

Their summation tree is the library's own, so they are held to what a plain dot in such
a tree must satisfy: the classical bound |dot - sum x_i y_i| <= gamma_m sum |x_i y_i|
(gamma_m = m u / (1 - m u), u the unit roundoff of the type), where m - 1 bounds the
number of additions any product passes through -- m = n for any order (used where
n u < 1), and for the documented tree (per-lane sums of at most c = ceil(n / lanes)
products over 512 * min(max(ceil(n / 4096), 1), 256) lanes, then 6 butterfly levels,
at most 8 wave additions, one exact start and 8 tree levels) m = c + 24; exactness on
small-integer inputs whose every partial sum is representable; reproducibility run to
run.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
from oracle import ctier
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def gamma(n, u):
    return n * u / (1 - n * u)


def tree_m(n):
    lanes = 512 * min(max(-(-n // 4096), 1), 256)
    return -(-n // lanes) + 24


@pytest.mark.parametrize("n", [1000, 1 << 20, 1 << 24])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_plain_dot_bound(n, dtype):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(dtype)
    y = (rng.standard_normal(n) * 10.0 ** rng.integers(-2, 3, n)).astype(dtype)
    tx, ty = to_dev(x), to_dev(y)
    got = pk.plain_dot(tx, ty)
    again = pk.plain_dot(tx, ty)
    assert torch.equal(got, again)
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    exact = ctier.exact_dot(x64, y64)
    u = 2.0 ** -24 if dtype == np.float32 else 2.0 ** -53
    absdot = ctier.exact_dot(np.abs(x64), np.abs(y64))
    err = abs(float(got.item()) - exact)
    # |exact| and sum |x y| are themselves rounded once (relative 2^-53): the slack
    m = min(n, tree_m(n))
    bound = gamma(m, u) * absdot * (1 + 2.0 ** -50)
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("n", [0, 1, 513, 4097, 1 << 20, 1 << 24])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_plain_dot_exact_on_integers(n, dtype):
    rng = np.random.default_rng(n + 3)
    lim = 1 if dtype == np.float32 else 1000
    x = rng.integers(-lim, lim + 1, n).astype(dtype)
    y = rng.integers(-lim, lim + 1, n).astype(dtype)
    exact = int(np.dot(x.astype(np.int64), y.astype(np.int64)))
    # every partial sum of any order is bounded by sum |x y|, below 2^24 / 2^53
    assert int(np.abs(x.astype(np.int64) * y.astype(np.int64)).sum()) < (2 ** 24 if dtype == np.float32 else 2 ** 53)
    got = pk.plain_dot(to_dev(x), to_dev(y)).item()
    assert got == exact


def test_plain_dot_invalid():
    x = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    import ctypes
    with pytest.raises(pk.LibError):
        rc = pk.lib().plain_dot(4, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 7,
                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 0, None)
        pk._check(rc, "plain_dot")
