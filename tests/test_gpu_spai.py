"""Learned SPAI kernels vs the float64 oracle (features, FP32 MLP forward, loss and
gradient, Adam, bf16 MFMA inference) and the gain of the trained preconditioner."""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import spai as ospai
from paper_2404_13216_amd import spai
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mat():
    p = g.problem("spai_eval_128", scale=14)
    return p


def rand_params(seed, scale=0.05):
    th = ospai.init_params(seed)
    th[4992:] = np.random.default_rng(seed + 1).standard_normal(65) * scale   # non-zero last layer
    return th


def test_features(mat):
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    got = sm.feat.view(-1, 12).cpu().numpy().astype(np.float64)
    ref = ospai.features(mat.A)
    err = np.abs(got - ref)
    assert np.all(err <= 1e-6 * np.abs(ref) + 1e-7), np.max(err / (np.abs(ref) + 1e-7))
    assert np.array_equal(sm.rowidx.cpu().numpy(), np.repeat(np.arange(mat.A.n), np.diff(mat.A.row_ptr)))
    assert np.array_equal(sm.diag.cpu().numpy(), mat.A.diag())


def test_features_hand_worked_unsymmetric():
    """All twelve features on the hand-worked unsymmetric 4 x 4 matrix of the oracle's
    pins (negative diagonal, a missing transpose entry), FP32 against the exact values."""
    from tests.test_oracle_spai import HAND_A, HAND_PHI
    rows = np.array([i for i, _, _ in HAND_A])
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=4))]).astype(np.int32)
    A = g.CSR(4, rp, np.array([j for _, j, _ in HAND_A], dtype=np.int32), np.array([v for _, _, v in HAND_A]))
    sm = spai.SpaiMatrix(pk.CSR.from_host(A))
    got = sm.feat.view(-1, 12).cpu().numpy().astype(np.float64)
    expect = np.array([[float(v) for v in row] for row in HAND_PHI])
    assert np.all(np.abs(got - expect) <= 2.0 ** -21 * np.abs(expect)), np.argwhere(got != expect)


def test_untrained_net_is_jacobi(mat):
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    th = torch.from_numpy(ospai.init_params(0).astype(np.float32)).cuda()
    rows = np.repeat(np.arange(mat.A.n), np.diff(mat.A.row_ptr))
    jac = np.where(rows == mat.A.col_idx, 1.0 / mat.A.diag()[rows], 0.0)
    for m in (sm.m_fp32(th), sm.m_bf16(th)):
        m = m.cpu().numpy().astype(np.float64)
        assert np.allclose(m, jac, rtol=2e-7, atol=0)


def test_forward_fp32(mat):
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    th = rand_params(3)
    m = sm.m_fp32(torch.from_numpy(th.astype(np.float32)).cuda()).cpu().numpy()
    ref = ospai.m_values(mat.A, th.astype(np.float32).astype(np.float64))
    rows = np.repeat(np.arange(mat.A.n), np.diff(mat.A.row_ptr))
    scale = 1.0 / np.abs(mat.A.diag()[rows])
    assert np.max(np.abs(m - ref) / scale) <= 1e-5


def test_bf16_inference_vs_emulation(mat):
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    th = rand_params(4, scale=0.2).astype(np.float32).astype(np.float64)
    m = sm.m_bf16(torch.from_numpy(th.astype(np.float32)).cuda()).cpu().numpy()
    ref = ospai.infer_bf16(mat.A, th)
    rows = np.repeat(np.arange(mat.A.n), np.diff(mat.A.row_ptr))
    inv = 1.0 / np.abs(mat.A.diag()[rows])
    assert np.all(np.abs(m - ref) <= 2.0 ** -7 * (np.abs(ref) + inv)), np.max(np.abs(m - ref) / (np.abs(ref) + inv))


def test_bf16_inference_wide_preactivations(mat):
    """Pre-activations far outside [-8, 8) (weights scaled up, large biases): the GELU
    table's first interval extended below -8 (G ~ 0) and its last one above 8 (G(z) = z)
    against the exact-GELU emulation."""
    th = rand_params(9, scale=0.05).astype(np.float32).astype(np.float64)
    W1, b1, W2, b2, w3, b3 = ospai.unpack(th)
    W1 *= 8.0
    b1[:] = np.random.default_rng(10).standard_normal(64) * 4.0
    W2 *= 1.5
    th = th.astype(np.float32).astype(np.float64)
    rows = np.repeat(np.arange(mat.A.n), np.diff(mat.A.row_ptr))
    phi = ospai.features(mat.A)
    # the emulation's pre-activations reach both extensions of the table (about -22 .. 21)
    W1, b1, W2, b2 = ospai.unpack(th)[:4]
    x0 = ospai.to_bf16(phi.astype(np.float32)).astype(np.float64)
    z1 = x0 @ ospai.to_bf16(W1.astype(np.float32)).astype(np.float64).T + b1
    h1 = ospai.to_bf16(ospai.gelu(z1).astype(np.float32)).astype(np.float64)
    z2 = h1 @ ospai.to_bf16(W2.astype(np.float32)).astype(np.float64).T + b2
    assert min(z1.min(), z2.min()) < -8.0 and min(z1.max(), z2.max()) > 8.0
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    m = sm.m_bf16(torch.from_numpy(th.astype(np.float32)).cuda()).cpu().numpy()
    ref = ospai.infer_bf16_values(th, phi, mat.A.diag()[rows])
    inv = 1.0 / np.abs(mat.A.diag()[rows])
    assert np.all(np.abs(m - ref) <= 2.0 ** -7 * (np.abs(ref) + inv)), np.max(np.abs(m - ref) / (np.abs(ref) + inv))


def test_bf16_inference_extreme_preactivations(mat):
    """Layer-1 pre-activations near +-1e4 (alternating huge biases): GELU must give z above
    the table and stay bounded near zero far below it."""
    th = rand_params(9, scale=0.05).astype(np.float32).astype(np.float64)
    b1 = ospai.unpack(th)[1]
    b1[:] = np.where(np.arange(64) % 2 == 0, 1.0e4, -1.0e4) * (1 + np.arange(64) / 64.0)
    th = th.astype(np.float32).astype(np.float64)
    rows = np.repeat(np.arange(mat.A.n), np.diff(mat.A.row_ptr))
    phi = ospai.features(mat.A)
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    m = sm.m_bf16(torch.from_numpy(th.astype(np.float32)).cuda()).cpu().numpy()
    ref = ospai.infer_bf16_values(th, phi, mat.A.diag()[rows])
    inv = 1.0 / np.abs(mat.A.diag()[rows])
    assert np.all(np.isfinite(m))
    assert np.all(np.abs(m - ref) <= 2.0 ** -7 * (np.abs(ref) + inv)), np.max(np.abs(m - ref) / (np.abs(ref) + inv))


def test_loss_grad_and_adam_step(mat):
    A = mat.A
    sm = spai.SpaiMatrix(pk.CSR.from_host(A))
    rng = np.random.default_rng(5)
    V = np.concatenate([g.rademacher(A.n, 4, 9), rng.standard_normal((A.n, 4))], axis=1).astype(np.float32)
    th = rand_params(6).astype(np.float32)
    Vc = torch.from_numpy(np.ascontiguousarray(V.T)).cuda()    # column-major n x k
    U = sm.probe_product(Vc, 8)
    p = torch.from_numpy(th).cuda()
    loss, grad = sm.loss_grad(p, Vc, U, 8)
    L, gref = ospai.loss_and_grad(A, th.astype(np.float64), V.astype(np.float64))
    gg = grad.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - L) <= 1e-4 * L
    assert np.linalg.norm(gg - gref) <= 1e-4 * np.linalg.norm(gref)
    # one Adam step
    mom = torch.zeros_like(p)
    vel = torch.zeros_like(p)
    spai.adam(p, mom, vel, grad, 1, lr=1e-3)
    tref, _, _ = ospai.adam_step(th.astype(np.float64), gg, np.zeros(5057), np.zeros(5057), 1, lr=1e-3)
    assert np.allclose(p.cpu().numpy(), tref, rtol=1e-6, atol=1e-9)


def test_gradient_deterministic(mat):
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    Vc = torch.from_numpy(np.ascontiguousarray(g.rademacher(mat.A.n, 8, 1).T.astype(np.float32))).cuda()
    U = sm.probe_product(Vc, 8)
    p = torch.from_numpy(rand_params(7).astype(np.float32)).cuda()
    g1 = sm.loss_grad(p, Vc, U, 8)[1].cpu().numpy()
    g2 = sm.loss_grad(p, Vc, U, 8)[1].cpu().numpy()
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32))


def test_trained_preconditioner_gains(capsys):
    """Train on small seeded matrices, evaluate on a held-out one: fewer iterations than
    the unpreconditioned solver (and report Jacobi)."""
    train = [g.training_problem(s, N=(18 if g.training_params(s)["dim"] == 3 else 64)) for s in range(100, 108)]
    params, hist = spai.train(train, epochs=25, lr=3e-3, seed=0)
    ev = g.problem("spai_eval_128", scale=24)
    A = pk.CSR.from_host(ev.A)
    b = to_dev(ev.b)
    sm = spai.SpaiMatrix(A)
    _, plain = pk.solve(A, b, tol=1e-10)
    _, jac = pk.solve(A, b, tol=1e-10, M=sm.preconditioner(spai.init_params(0)))
    _, learned = pk.solve(A, b, tol=1e-10, M=sm.preconditioner(params), fallback=1)
    with capsys.disabled():
        print(f"\n  loss {hist[0]:.4e} -> {hist[-1]:.4e}; iterations plain {plain['iterations']} "
              f"jacobi {jac['iterations']} learned {learned['iterations']} (fell back {learned['fell_back']})")
    assert hist[-1] < hist[0]
    assert learned["status"] == pk.OK and learned["true_relres"] <= 1e-10
    assert learned["iterations"] < plain["iterations"]


def test_train_step_equals_loss_grad_then_adam(mat):
    """spai_train_step = spai_loss_grad followed by spai_adam, bit for bit."""
    sm = spai.SpaiMatrix(pk.CSR.from_host(mat.A))
    Vc = torch.from_numpy(np.ascontiguousarray(g.rademacher(mat.A.n, 8, 2).T.astype(np.float32))).cuda()
    U = sm.probe_product(Vc, 8)
    p0 = torch.from_numpy(rand_params(9).astype(np.float32)).cuda()
    pa, pb = p0.clone(), p0.clone()
    ma, va = torch.zeros_like(p0), torch.zeros_like(p0)
    mb, vb = torch.zeros_like(p0), torch.zeros_like(p0)
    for t in (1, 2):
        loss_a, grad = sm.loss_grad(pa, Vc, U, 8)
        spai.adam(pa, ma, va, grad, t, lr=1e-3)
        loss_b = sm.train_step(pb, mb, vb, Vc, U, 8, t, lr=1e-3)
        assert loss_a.item() == loss_b.item()
    assert torch.equal(pa.view(torch.int32), pb.view(torch.int32))
    assert torch.equal(ma.view(torch.int32), mb.view(torch.int32))


def test_probe_block_vs_oracle():
    """The training probe block: Rademacher columns as drawn, residual columns
    r_i / ||r_i|| (norm from the exact dot, rounded to FP32 once) bit for bit against the
    oracle's probe block (the GPU residuals are bit-identical to the oracle's)."""
    p = g.problem("spai_eval_128", scale=12)
    A = pk.CSR.from_host(p.A)
    Vc = spai.probe_block(A, to_dev(p.b), seed=77).cpu().numpy()
    ref = ospai.probe_block(p.A, p.b, seed=77).astype(np.float32)
    assert Vc.shape == (8, p.A.n)
    assert np.array_equal(Vc.view(np.uint32), np.ascontiguousarray(ref.T).view(np.uint32))
    # a zero residual gives a zero column
    z = torch.zeros(5, dtype=torch.float64, device="cuda:0")
    out = torch.full((5,), 7.0, dtype=torch.float32, device="cuda:0")
    ws = torch.empty(pk.lib().spai_probe_column_workspace_bytes(5), dtype=torch.uint8, device="cuda:0")
    import ctypes
    rc = pk.lib().spai_probe_column(5, ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0 and not out.any()
