"""FP32-inner / FP64-refinement solve on the GPU vs the FP64 oracle.

The inner solver runs in FP32 with plain FP32 dots (the GPU reduces them in a
fixed tree, the oracle sequentially), so inner trajectories differ; the bar is that
both reach the true relative residual 1e-10 and that the refined solution agrees
with the FP64 oracle's to the accuracy the residual implies.  The error against the
FP64 oracle is reported per case.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier, solvers
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,scale", [("cd3d_128", 32), ("rand_1m", 30000), ("cd3d_256_var", 24),
                                        ("cd2d_64", None)])
def test_ir_reaches_1e10(name, scale, capsys):
    p = g.problem(name, scale=scale)
    ref = ctier.pbicgstab(p.A, p.b, tol=1e-10, max_iter=20000)  # the FP64 oracle at the same tolerance
    assert ref["status"] == 0
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-10, prec=pk.PREC_FP32_IR, max_iter=5000)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    assert info["status"] == pk.OK and info["true_relres"] <= 1e-10, info
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    err_star = np.linalg.norm(x - p.xstar) / np.linalg.norm(p.xstar)
    ora = solvers.ir_solve(p.A, p.b, tol=1e-10)
    with capsys.disabled():
        print(f"\n  {name}: outer {info['outer_iterations']} inner {info['iterations']} "
              f"true {info['true_relres']:.2e} err_vs_fp64_oracle {err:.2e} err_vs_xstar {err_star:.2e}; "
              f"oracle IR outer {ora.outer_iterations} inner {ora.iterations} status {ora.status}")
    assert ora.status == solvers.OK
    assert err <= 1e-6


def test_ir_zero_rhs_and_invalid():
    p = g.problem("cd2d_64", scale=8)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(np.zeros(p.A.n)), prec=pk.PREC_FP32_IR)
    assert info["status"] == pk.OK and not x.any()
    with pytest.raises(pk.LibError):
        pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), prec=pk.PREC_FP32_IR, alg=pk.ALG_BICGSTAB)
