"""The allocation-free exact dot (exdot_noalloc, for callers that cannot allocate) returns
the same bits as exdot on the same inputs, on consecutive calls that share the library's
static scratch array -- the second call with a smaller input, so stale records of the
first would show -- and both equal the oracle's exact dot."""
import ctypes

import numpy as np
import pytest

import paper_2404_13216_amd as pk
from oracle import ctier
import synthgen as g
from tests.gpu_util import same_bits, to_dev

pytestmark = pytest.mark.gpu


def _call_noalloc(x, y, out):
    import torch
    rc = pk.lib().exdot_noalloc(x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == pk.OK, pk.status_string(rc)


@pytest.mark.parametrize("sizes", [(3_000_000, 70_001), (2 ** 22 + 17, 1), (4096 * 512 * 3, 0)])
def test_noalloc_matches_exdot_twice(sizes):
    import torch
    out = torch.empty(1, dtype=torch.float64, device="cuda:0")
    for k, n in enumerate(sizes):
        xs = g.wide_exponent_vec(n, 100 + k, emin=-600, emax=600)
        ys = g.uniform_vec(n, 300 + k)
        x, y = to_dev(xs), to_dev(ys)
        _call_noalloc(x, y, out)
        got = out.item()
        ref = pk.exdot(x, y).item()
        torch.cuda.synchronize()
        assert same_bits(got, ref), (n, got, ref)
        assert same_bits(got, ctier.exact_dot(xs, ys)), (n, got)


def test_noalloc_rejects_oversize_without_launch():
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    x = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    rc = pk.lib().exdot_noalloc((1 << 34) + 1, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == pk.ERR_INVALID
    assert pk.lib().exdot_noalloc_scratch_bytes() < (1 << 20)
