"""The comparators of the paper's central claim on the GPU, against the oracle.

Ordinary FP64 dots run in a fixed reduction tree that the oracle defines identically,
and the residual replacement is a fixed sequence of row-sequential SpMVs, so both
comparators are compared bit for bit: same iterate, same recursive-residual history,
same iteration count.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import solvers
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def run_both(p, dots, rr, tol=1e-10, max_iter=3000):
    ex = solvers.default_dot(p.A.n)
    dot = solvers.dot_f64_tree if dots == pk.DOTS_PLAIN else ex
    ref = solvers.pbicgstab(p.A, p.b, tol=tol, max_iter=max_iter, dot=dot, exact_dot=ex, rr_period=rr)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=tol, max_iter=max_iter, dots=dots, rr_period=rr,
                       history=max_iter)
    torch.cuda.synchronize()
    return ref, x.cpu().numpy(), info


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 24), ("rand_1m", 8000),
                                        ("cd3d_256_var", 20)])
@pytest.mark.parametrize("dots,rr", [(pk.DOTS_PLAIN, 0), (pk.DOTS_EXACT, 10), (pk.DOTS_PLAIN, 7)])
def test_comparator_bitwise(name, scale, dots, rr):
    p = g.problem(name, scale=scale)
    ref, x, info = run_both(p, dots, rr)
    assert info["status"] == ref.status
    assert info["iterations"] == ref.iterations
    assert np.array_equal(bits(info["history"]), bits(ref.history))
    assert np.array_equal(bits(x), bits(ref.x))
    assert info["true_relres"] == ref.true_relres


def test_comparator_invalid_combinations():
    p = g.problem("cd2d_64", scale=8)
    A, b = pk.CSR.from_host(p.A), to_dev(p.b)
    for kw in ({"dots": pk.DOTS_PLAIN, "alg": pk.ALG_BICGSTAB}, {"rr_period": 5, "prec": pk.PREC_FP32_IR},
               {"dots": 7}, {"rr_period": -1}):
        with pytest.raises(pk.LibError):
            pk.solve(A, b, **kw)


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 24)])
@pytest.mark.parametrize("dots", [pk.DOTS_EXACT, pk.DOTS_PLAIN])
def test_true_history_bitwise(name, scale, dots):
    """The recursive / true residual gap past the attainable accuracy (tol 1e-13): the
    true residual every 10 iterations, bit for bit with the oracle."""
    p = g.problem(name, scale=scale)
    ex = solvers.default_dot(p.A.n)
    dot = solvers.dot_f64_tree if dots == pk.DOTS_PLAIN else ex
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-13, max_iter=300, dot=dot, exact_dot=ex, true_every=10)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-13, max_iter=300, dots=dots, true_every=10,
                       history=300)
    assert info["iterations"] == ref.iterations and info["true_checks"] == ref.true_checks
    assert len(info["true_history"]) == len(ref.true_history) > 0
    assert np.array_equal(bits(info["true_history"]), bits(ref.true_history))
    assert np.array_equal(bits(info["history"]), bits(ref.history))
