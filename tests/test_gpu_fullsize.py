"""Parity at the full sizes of the workloads, in the launch configuration the bench
times: whole vectors where the oracle is fast enough, sampled rows / nonzeros (each
computed one by one in the oracle's order) otherwise.

* random 10^6 (17.8M nonzeros, rows up to 400): FP64 SpMV and the Dot2 FP32 SpMV bit
  for bit on every row; 20 p-BiCGStab iterations bit for bit against the C oracle.
* 256^3 variable diffusivity (117M nonzeros): both SpMVs bit for bit on 20,000 sampled
  rows; 5 p-BiCGStab iterations bit for bit against the C oracle (the solve's sliced copy,
  1.4 GB, is larger than the Infinity Cache and is read with non-temporal loads).
* held-out 128^3 learned-preconditioner matrix: features on every nonzero against the
  float64 oracle; bf16 inference against the oracle's emulation on 50,000 sampled
  nonzeros.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier
from oracle import spai as ospai
from oracle.spmv import spmv, spmv_f32, spmv_f32_loops, spmv_loops
from paper_2404_13216_amd import spai
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def sub_rows(A, rows, dtype=np.float64):
    """The CSR of the given rows (columns and values unchanged)."""
    lens = np.diff(A.row_ptr.astype(np.int64))[rows]
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in rows])
    return g.CSR(len(rows), rp.astype(np.int32), A.col_idx[idx], A.val[idx].astype(dtype))


def gpu_solve_iters(p, its):
    Ad = pk.CSR.from_host(p.A)
    x, info = pk.solve(Ad, to_dev(p.b), tol=1e-10, max_iter=its)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


def test_rand_1m_full():
    p = g.problem("rand_1m")
    A = p.A
    x = np.random.default_rng(11).uniform(-1, 1, A.n)
    Ad = pk.CSR.from_host(A)
    y = pk.csr_spmv(Ad, to_dev(x)).cpu().numpy()
    assert np.array_equal(bits(y), bits(spmv(A, x)))
    A32 = g.CSR(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32))
    x32 = x.astype(np.float32)
    y32 = pk.csr_spmv_f32(pk.CSR.from_host(A, dtype=torch.float32), to_dev(x32)).cpu().numpy()
    assert np.array_equal(y32.view(np.uint32), spmv_f32(A32, x32).view(np.uint32))
    ora = ctier.pbicgstab(A, p.b, tol=1e-10, max_iter=20)
    xg, info = gpu_solve_iters(p, 20)
    assert info["iterations"] == ora["iterations"] == 20
    assert np.array_equal(bits(xg), bits(ora["x"]))


def test_cd3d_256_full_sampled():
    p = g.problem("cd3d_256_var")
    A = p.A
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, A.n)
    rows = np.sort(rng.choice(A.n, 20000, replace=False))
    rows[:2] = [0, A.n - 1]
    Ad = pk.CSR.from_host(A)
    y = pk.csr_spmv(Ad, to_dev(x)).cpu().numpy()
    S = sub_rows(A, rows)
    assert np.array_equal(bits(y[rows]), bits(spmv_loops(S, x)))
    x32 = x.astype(np.float32)
    y32 = pk.csr_spmv_f32(pk.CSR.from_host(A, dtype=torch.float32), to_dev(x32)).cpu().numpy()
    S32 = sub_rows(A, rows, np.float32)
    assert np.array_equal(y32[rows].view(np.uint32), np.array(spmv_f32_loops(S32, x32), dtype=np.float32).view(np.uint32))
    del Ad
    ora = ctier.pbicgstab(A, p.b, tol=1e-10, max_iter=5)
    xg, info = gpu_solve_iters(p, 5)
    assert info["iterations"] == ora["iterations"] == 5
    assert np.array_equal(bits(xg), bits(ora["x"]))


def test_spai_eval_full_features_and_inference():
    p = g.problem("spai_eval_128")
    A = p.A
    sm = spai.SpaiMatrix(pk.CSR.from_host(A))
    feat = sm.feat.view(A.nnz, 12).cpu().numpy().astype(np.float64)
    phi = ospai.features(A)
    assert np.all(np.abs(feat - phi) <= 1e-6 * np.abs(phi) + 1e-7)
    rng = np.random.default_rng(13)
    th = ospai.init_params(21)
    th[4992:] = rng.standard_normal(65) * 0.2
    th32 = th.astype(np.float32)
    m = sm.m_bf16(torch.from_numpy(th32).cuda()).cpu().numpy()
    pick = rng.choice(A.nnz, 50000, replace=False)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    aii = A.diag()[rows[pick]]
    ref = ospai.infer_bf16_values(th32.astype(np.float64), phi[pick], aii)
    inv = 1.0 / np.abs(aii)
    assert np.all(np.abs(m[pick] - ref) <= 2.0 ** -7 * (np.abs(ref) + inv))
