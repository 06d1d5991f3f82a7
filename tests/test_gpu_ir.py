"""FP32 refinement with reliable updates on the GPU vs the oracle.

Every piece of the GPU solve has a bit-exact counterpart in the oracle: the FP64
row-sequential SpMV and exact dots of the reliable updates, the compensated FP32 SpMV,
the FP32 dots in their fixed reduction tree, and the FP32 recurrences and scalars in the
same order with separate roundings.  The solves are therefore compared bit for bit:
same iterate, same FP32 iteration count, same number of reliable updates.  The error of
the refined solution against the FP64 oracle's is reported per case.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier, solvers
from oracle.spmv import spmv_f32
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,scale", [("cd2d_64", 20), ("cd2d_64", None), ("cd3d_128", 24),
                                        ("cd3d_256_var", 20), ("rand_1m", 8000), ("spai_eval_128", 16)])
def test_ir_bitwise(name, scale, capsys):
    p = g.problem(name, scale=scale)
    ora = solvers.ir_solve(p.A, p.b, tol=1e-10, max_iter=5000)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-10, prec=pk.PREC_FP32_IR, max_iter=5000)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    ref = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=20000)
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    with capsys.disabled():
        print(f"\n  {name}/{scale}: updates {info['outer_iterations']} FP32 iterations {info['iterations']} "
              f"(FP64 solve {ref['iterations']}) fell back {info['fell_back']} true {info['true_relres']:.2e} "
              f"err vs FP64 oracle {err:.2e}")
    assert ora.status == solvers.OK and info["status"] == pk.OK
    assert info["true_relres"] <= 1e-10
    assert info["iterations"] == ora.iterations
    assert info["outer_iterations"] == ora.outer_iterations
    assert info["fell_back"] == ora.fell_back
    assert np.array_equal(x.view(np.uint64), ora.x.view(np.uint64))


def test_ir_finish_path_bitwise():
    """max_outer = 1: one reliable update, then the FP64 finish from the best iterate."""
    p = g.problem("cd3d_256_var", scale=16)
    ora = solvers.ir_solve(p.A, p.b, tol=1e-10, max_iter=5000, max_outer=1)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-10, prec=pk.PREC_FP32_IR, max_iter=5000,
                       max_outer=1)
    assert ora.fell_back == 1 and info["fell_back"] == 1
    assert info["status"] == ora.status == pk.OK
    assert info["iterations"] == ora.iterations
    assert np.array_equal(x.cpu().numpy().view(np.uint64), ora.x.view(np.uint64))


def test_csr_spmv_f32_dot2_bitwise():
    for name, scale in (("rand_1m", 3000), ("cd3d_256_var", 24)):
        p = g.problem(name, scale=scale)
        A32 = g.CSR(p.A.n, p.A.row_ptr, p.A.col_idx, p.A.val.astype(np.float32))
        x = np.random.default_rng(5).uniform(-1, 1, p.A.n).astype(np.float32)
        y = pk.csr_spmv_f32(pk.CSR.from_host(p.A, dtype=torch.float32), to_dev(x)).cpu().numpy()
        assert np.array_equal(y.view(np.uint32), spmv_f32(A32, x).view(np.uint32))


def test_ir_zero_rhs_and_invalid():
    p = g.problem("cd2d_64", scale=8)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(np.zeros(p.A.n)), prec=pk.PREC_FP32_IR)
    assert info["status"] == pk.OK and not x.any()
    with pytest.raises(pk.LibError):
        pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), prec=pk.PREC_FP32_IR, alg=pk.ALG_BICGSTAB)
