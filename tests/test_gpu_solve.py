"""Whole-solve parity of the GPU p-BiCGStab / BiCGStab against the oracle.

With the default row-sequential SpMV every operation of the GPU solve rounds exactly
as the oracle's does (exact dots rounded once, literal-order updates, left-to-right
row sums), so iterates, residuals, iteration counts and true residuals are
bit-identical, which meets the bar ||x_i^gpu - x_i^orc|| / ||x_i^orc|| <= 1e-12 for the
first 20 iterations with room to spare.  The tree-ordered SpMV kernels (vector CSR,
wavefront per row) round differently; they do NOT meet that bar everywhere: on the 64^2
workload their iterates drift to 6.5e-12 by iteration 17.  They are held, iteration by
iteration for the first 20, to 1e-10 (the maximum is printed), and must reach the true
relative residual 1e-10 like the oracle.
"""
import math

import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier, solvers
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu


def gpu_solve(A, b, r_out=False, **kw):
    Ad = pk.CSR.from_host(A)
    bd = to_dev(b)
    s = pk.Solver(Ad, **kw)
    r = torch.empty(A.n, dtype=torch.float64, device=dev()) if r_out else None
    x, info = s.solve(bd, None, r_out=r)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info, (r.cpu().numpy() if r_out else None)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("alg", [pk.ALG_PBICGSTAB, pk.ALG_BICGSTAB])
def test_twenty_iterations_bit_identical_cd2d(alg):
    p = g.problem("cd2d_64")
    f = solvers.pbicgstab if alg == pk.ALG_PBICGSTAB else solvers.bicgstab
    ref = f(p.A, p.b, tol=1e-10, max_iter=20, record=20)
    assert len(ref.iterates) == 20
    for i in range(1, 21):
        x, info, r = gpu_solve(p.A, p.b, r_out=True, tol=1e-10, max_iter=i, alg=alg)
        assert info["iterations"] == i and info["status"] == pk.NOT_CONVERGED
        xo, ro, _, _ = ref.iterates[i - 1]
        assert np.array_equal(bits(x), bits(xo)), i
        assert np.array_equal(bits(r), bits(ro)), i


@pytest.mark.parametrize("alg", [pk.ALG_PBICGSTAB, pk.ALG_BICGSTAB])
def test_converges_cd2d(alg):
    p = g.problem("cd2d_64")
    f = ctier.pbicgstab if alg == pk.ALG_PBICGSTAB else ctier.bicgstab
    ref = f(p.A, p.b, tol=1e-10, max_iter=2000)
    x, info, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=2000, alg=alg, history=0)
    assert info["status"] == pk.OK and info["true_relres"] <= 1e-10
    assert ref["status"] == 0 and ref["true_relres"] <= 1e-10
    assert info["iterations"] == ref["iterations"] and info["true_checks"] == ref["true_checks"]
    assert bits(info["true_relres"]) == bits(ref["true_relres"])
    assert np.array_equal(bits(x), bits(ref["x"]))
    assert rel(x, p.xstar) <= 1e-6
    # tree-ordered SpMV kernels: same bar on convergence
    for kind in (pk.SPMV_VECTOR, pk.SPMV_WAVE):
        xv, iv, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=2000, alg=alg, spmv_kind=kind)
        assert iv["status"] == pk.OK and iv["true_relres"] <= 1e-10
        assert rel(xv, ref["x"]) <= 1e-8


@pytest.mark.parametrize("name", ["cd2d_64", "cd3d_128"])
@pytest.mark.parametrize("kind", [pk.SPMV_VECTOR, pk.SPMV_WAVE])
def test_tree_kinds_first_twenty(name, kind, capsys):
    """Tree-ordered SpMV kinds, every one of the first 20 iterates against the oracle's."""
    p = g.problem(name)
    worst = 0.0
    for i in range(1, 21):
        ora = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=i)
        x, info, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=i, spmv_kind=kind)
        assert info["iterations"] == i == ora["iterations"]
        worst = max(worst, rel(x, ora["x"]))
    with capsys.disabled():
        print(f"\n  {name} kind {kind}: max relative iterate difference over 20 iterations {worst:.2e}")
    assert worst <= 1e-10


def test_history_matches_oracle_early():
    p = g.problem("cd2d_64")
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-10, max_iter=2000)
    Ad, bd = pk.CSR.from_host(p.A), to_dev(p.b)
    x, info = pk.solve(Ad, bd, history=2000, tol=1e-10, max_iter=2000)
    h = info["history"]
    assert len(h) == len(ref.history)
    assert np.array_equal(bits(h), bits(ref.history))


@pytest.mark.parametrize("name,scale", [("cd3d_128", 32), ("rand_1m", 30000), ("cd3d_256_var", 24)])
def test_converges_other_families(name, scale):
    p = g.problem(name, scale=scale)
    ref = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=5000)
    x, info, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=5000)
    assert info["status"] == pk.OK and info["true_relres"] <= 1e-10, info
    assert ref["status"] == 0
    assert info["iterations"] == ref["iterations"]
    assert np.array_equal(bits(x), bits(ref["x"]))
    refb = ctier.bicgstab(p.A, p.b, tol=1e-10, max_iter=5000)
    xb, infob, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=5000, alg=pk.ALG_BICGSTAB)
    assert infob["iterations"] == refb["iterations"] and np.array_equal(bits(xb), bits(refb["x"]))


def test_full_size_128_parity_and_convergence():
    """The 128^3 workload (n = 2,097,152): 20-iteration parity, then the full solve."""
    p = g.problem("cd3d_128")
    ora = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=20)
    x20, info, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=20)
    assert info["iterations"] == 20 == ora["iterations"]
    assert np.array_equal(bits(x20), bits(ora["x"]))
    xv, infov, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=20, spmv_kind=pk.SPMV_VECTOR)
    assert rel(xv, ora["x"]) <= 1e-12
    x, info, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=10000)
    assert info["status"] == pk.OK and info["true_relres"] <= 1e-10, info
    xb, infob, _ = gpu_solve(p.A, p.b, tol=1e-10, max_iter=10000, alg=pk.ALG_BICGSTAB)
    assert infob["status"] == pk.OK and infob["true_relres"] <= 1e-10, infob


def test_run_to_run_bitwise_solve():
    p = g.problem("rand_1m", scale=20000)
    x1, i1, _ = gpu_solve(p.A, p.b, tol=1e-10)
    x2, i2, _ = gpu_solve(p.A, p.b, tol=1e-10)
    assert i1["iterations"] == i2["iterations"]
    assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))


# ------------------------------------------------------------------ special cases
def csr_dense(D):
    import scipy.sparse as sp
    S = sp.csr_matrix(D)
    S.sort_indices()
    return g.CSR(D.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


@pytest.mark.parametrize("alg", [pk.ALG_PBICGSTAB, pk.ALG_BICGSTAB])
def test_identity_lucky_breakdown(alg):
    A = csr_dense(np.eye(33))
    b = np.random.default_rng(0).standard_normal(33)
    x, info, _ = gpu_solve(A, b, alg=alg)
    assert info["status"] == pk.OK and info["iterations"] == 1
    assert np.array_equal(x, b)


def test_skew_breakdown():
    rng = np.random.default_rng(1)
    K = np.triu(rng.integers(-4, 5, (12, 12)).astype(float), 1)
    A = csr_dense(K - K.T)
    b = rng.integers(-3, 4, 12).astype(float)
    x, info, _ = gpu_solve(A, b)
    assert info["status"] == pk.BREAKDOWN and info["iterations"] == 0
    assert solvers.pbicgstab(A, b).status == solvers.BREAKDOWN


def test_zero_rhs_nan_rhs_and_limits():
    p = g.problem("cd2d_64", scale=16)
    x, info, _ = gpu_solve(p.A, np.zeros(p.A.n))
    assert info["status"] == pk.OK and info["iterations"] == 0 and not x.any()
    bn = p.b.copy()
    bn[5] = math.nan
    x, info, _ = gpu_solve(p.A, bn)
    assert info["status"] == pk.ERR_NONFINITE
    x, info, _ = gpu_solve(p.A, p.b, tol=0.0, max_iter=7)
    ref = solvers.pbicgstab(p.A, p.b, tol=0.0, max_iter=7)
    assert info["status"] == ref.status and info["iterations"] == ref.iterations
    x, info, _ = gpu_solve(p.A, p.b, max_iter=0)
    assert info["status"] == pk.NOT_CONVERGED and info["iterations"] == 0


def test_warm_start_exact_solution():
    p = g.problem("cd2d_64", scale=16)
    Ad, bd = pk.CSR.from_host(p.A), to_dev(p.b)
    x0 = torch.from_numpy(np.linalg.solve(p.A.to_scipy().toarray(), p.b)).to(dev())
    x, info = pk.solve(Ad, bd, x0=x0, tol=1e-10)
    assert info["status"] == pk.OK and info["iterations"] == 0


@pytest.mark.parametrize("name,scale", [("cd2d_64", None), ("cd3d_128", 32), ("rand_1m", 20000)])
def test_stagnation_rule_bitwise(name, scale):
    """Tolerance 1e-14, below what p-BiCGStab's recurrences sustain: the failed true-residual
    tests, the STAGNATED status and the returned (best tested) iterate match the oracle bit
    for bit; BiCGStab reaches the tolerance on both sides."""
    p = g.problem(name, scale=scale)
    ora = ctier.pbicgstab(p.A, p.b, tol=1e-14, max_iter=3000)
    x, info, _ = gpu_solve(p.A, p.b, tol=1e-14, max_iter=3000)
    assert info["status"] == ora["status"] == pk.STAGNATED
    assert info["iterations"] == ora["iterations"] and info["true_checks"] == ora["true_checks"]
    assert np.array_equal(bits(x), bits(ora["x"])) and info["true_relres"] == ora["true_relres"]
    orb = ctier.bicgstab(p.A, p.b, tol=1e-14, max_iter=3000)
    xb, infob, _ = gpu_solve(p.A, p.b, tol=1e-14, max_iter=3000, alg=pk.ALG_BICGSTAB)
    assert infob["status"] == orb["status"] == pk.OK and np.array_equal(bits(xb), bits(orb["x"]))


def test_kernel_events_leave_the_solve_unchanged():
    """Timing events stamped by the kernels' own dispatches (a measurement option) change
    nothing: same iterate bits as the oracle's and as an untimed solve; every timed kernel
    has a positive duration shorter than the whole solve."""
    p = g.problem("cd3d_128", scale=48)
    ref = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=10000)
    x0, i0, _ = gpu_solve(p.A, p.b, tol=1e-10)
    Ad = pk.CSR.from_host(p.A)
    s = pk.Solver(Ad, kernel_events=16, tol=1e-10)
    x1, i1 = s.solve(to_dev(p.b))
    x1 = x1.cpu().numpy()
    assert i1["status"] == i0["status"] == pk.OK and i1["iterations"] == i0["iterations"] == ref["iterations"]
    assert np.array_equal(bits(x1), bits(x0))
    assert np.array_equal(bits(x1), bits(ref["x"]))
    kt = s.kernel_times()
    assert set(kt) == set(pk.Solver.KERNELS)
    for name, ts in kt.items():
        assert len(ts) == 16
        assert all(0.0 < t < i1["seconds"] for t in ts), (name, ts)
