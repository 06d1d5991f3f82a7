"""The comparators of the paper's central claim on the GPU, against the oracle.

* Residual replacement with exact dots is a fixed sequence of row-sequential SpMVs and
  exact dots, so it is compared bit for bit: same iterate, same recursive-residual
  history, same iteration count.
* Ordinary FP64 dots are formed in the library's fixed reduction tree; the oracle's
  ordinary dot is the sequential sum of its definition, so those runs differ by rounding
  (and the Krylov process amplifies the difference).  They are judged by outcome
  (tests/outcome.py): converged, the true residual recomputed by the oracle at or below
  the tolerance and equal to the reported one, the iterate within the certified
  perturbation bound of the oracle's exact-dot solution; the run is reproducible bit
  for bit, and its true-residual history matches, bit for bit, the oracle's true
  residual of the GPU's own iterates at those iterations.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import solvers
from tests import outcome as oc
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


CASES = [("cd2d_64", None), ("cd3d_128", 24), ("rand_1m", 8000), ("cd3d_256_var", 20)]


@pytest.mark.parametrize("name,scale", CASES)
def test_replacement_exact_bitwise(name, scale):
    p = g.problem(name, scale=scale)
    ex = solvers.default_dot(p.A.n)
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-10, max_iter=3000, dot=ex, rr_period=10)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-10, max_iter=3000, rr_period=10, history=3000)
    x = x.cpu().numpy()
    assert info["status"] == ref.status
    assert info["iterations"] == ref.iterations
    assert np.array_equal(bits(info["history"]), bits(ref.history))
    assert np.array_equal(bits(x), bits(ref.x))
    assert info["true_relres"] == ref.true_relres


@pytest.mark.parametrize("name,scale", CASES)
@pytest.mark.parametrize("rr", [0, 7])
def test_plain_dots_outcome(name, scale, rr, capsys):
    p = g.problem(name, scale=scale)
    A, b = pk.CSR.from_host(p.A), to_dev(p.b)
    x, info = pk.solve(A, b, tol=1e-10, max_iter=3000, dots=pk.DOTS_PLAIN, rr_period=rr)
    x2, info2 = pk.solve(A, b, tol=1e-10, max_iter=3000, dots=pk.DOTS_PLAIN, rr_period=rr)
    assert torch.equal(x.view(torch.int64), x2.view(torch.int64)) and info["iterations"] == info2["iterations"]
    x = x.cpu().numpy()
    ex = solvers.default_dot(p.A.n)
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-10, max_iter=3000, dot=ex)
    pl = solvers.pbicgstab(p.A, p.b, tol=1e-10, max_iter=3000, dot=solvers.dot_f64_seq, exact_dot=ex, rr_period=rr)
    true = oc.true_relres(p.A, p.b, x)
    gap = float(np.abs(x - ref.x).max())
    bound = oc.solution_gap_bound(p.A, p.b, x, ref.x)
    with capsys.disabled():
        print(f"\n  {name}/{scale} rr {rr}: GPU plain dots {info['iterations']} it, oracle plain "
              f"{pl.iterations}, exact {ref.iterations}; true {true:.2e}; |x - x_exact|_inf {gap:.2e} "
              f"(bound {bound:.2e})")
    assert info["status"] == pk.OK and ref.status == solvers.OK
    assert true <= 1e-10 and true == info["true_relres"]
    assert gap <= bound


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 24)])
def test_true_history_exact_bitwise(name, scale):
    """The recursive / true residual gap past the attainable accuracy (tol 1e-13): the
    true residual every 10 iterations, bit for bit with the oracle."""
    p = g.problem(name, scale=scale)
    ex = solvers.default_dot(p.A.n)
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-13, max_iter=300, dot=ex, true_every=10)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-13, max_iter=300, true_every=10, history=300)
    assert info["iterations"] == ref.iterations and info["true_checks"] == ref.true_checks
    assert len(info["true_history"]) == len(ref.true_history) > 0
    assert np.array_equal(bits(info["true_history"]), bits(ref.true_history))
    assert np.array_equal(bits(info["history"]), bits(ref.history))


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 24)])
def test_true_history_plain(name, scale):
    """With ordinary dots: every recorded true residual is the oracle's true residual of
    the GPU's own iterate at that iteration (a solve cut off there returns it; the
    fixed tree makes the runs identical up to the cut)."""
    p = g.problem(name, scale=scale)
    A, b = pk.CSR.from_host(p.A), to_dev(p.b)
    x, info = pk.solve(A, b, tol=1e-13, max_iter=300, dots=pk.DOTS_PLAIN, true_every=10)
    th = info["true_history"]
    assert len(th) >= 3
    for k in (1, 2, 3):
        xk, ik = pk.solve(A, b, tol=1e-13, max_iter=10 * k, dots=pk.DOTS_PLAIN)
        assert ik["iterations"] == 10 * k
        assert oc.true_relres(p.A, p.b, xk.cpu().numpy()) == th[k - 1], k


def test_comparator_invalid_combinations():
    p = g.problem("cd2d_64", scale=8)
    A, b = pk.CSR.from_host(p.A), to_dev(p.b)
    for kw in ({"dots": pk.DOTS_PLAIN, "alg": pk.ALG_BICGSTAB}, {"rr_period": 5, "prec": pk.PREC_FP32_IR},
               {"dots": 7}, {"rr_period": -1}):
        with pytest.raises(pk.LibError):
            pk.solve(A, b, **kw)
