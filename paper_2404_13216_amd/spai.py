"""Learned sparse approximate inverse: binding of the spai_* C-ABI calls plus the host
training loop (argument marshalling and loop control only; every arithmetic step runs
in the HIP kernels of libpbicgstab.so).

m_ij = ([i == j] + f(phi_ij)) / a_ii on A's pattern; f is an MLP 12 -> 64 -> 64 -> 1
(GELU).  Training minimises ||M A V - V||_F^2 / (k n) over probe blocks V built from
Rademacher columns and normalised residuals of plain p-BiCGStab runs on the training
matrix; inference runs in bf16 on the matrix cores and the result is applied as a right
preconditioner (opts.M) with the unpreconditioned solver as fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import CSR, Solver, _check, _ptr, _stream, _workspace, lib, solve

NPARAM = 5057


def _torch():
    import torch
    return torch


class SpaiMatrix:
    """A (FP64 CSR on the device) with its features, row indices and diagonal."""

    def __init__(self, A: CSR, k_max: int = 8, ws=None):
        """`ws`: optional shared device workspace of at least workspace_bytes(A, k_max)
        bytes (training shares one across its matrices; calls on one stream only)."""
        torch = _torch()
        dev = A.val.device
        self.A = A
        self.feat = torch.empty(A.nnz * 12, dtype=torch.float32, device=dev)
        self.rowidx = torch.empty(A.nnz, dtype=torch.int32, device=dev)
        self.diag = torch.empty(A.n, dtype=torch.float64, device=dev)
        need = workspace_bytes(A, k_max)
        if ws is not None and ws.numel() < need:
            raise ValueError(f"shared workspace too small: {ws.numel()} < {need}")
        self.ws = ws if ws is not None else _workspace(need, dev)
        self.k_max = k_max
        _check(lib().spai_features(A.c, _ptr(self.feat), _ptr(self.rowidx), _ptr(self.diag), _ptr(self.ws),
                                   self.ws.numel(), _stream()), "spai_features")

    def m_fp32(self, params, f_out=None):
        torch = _torch()
        m = torch.empty(self.A.nnz, dtype=torch.float32, device=params.device)
        _check(lib().spai_forward(self.A.nnz, _ptr(self.feat), _ptr(params), _ptr(self.rowidx), _ptr(self.A.col_idx),
                                  _ptr(self.diag), _ptr(f_out), _ptr(m), _stream()), "spai_forward")
        return m

    def m_bf16(self, params):
        torch = _torch()
        m = torch.empty(self.A.nnz, dtype=torch.float32, device=params.device)
        _check(lib().spai_infer_bf16(self.A.nnz, _ptr(self.feat), _ptr(params), _ptr(self.rowidx), _ptr(self.diag),
                                     _ptr(m), _stream()), "spai_infer_bf16")
        return m

    def preconditioner(self, params, bf16: bool = True) -> CSR:
        m = self.m_bf16(params) if bf16 else self.m_fp32(params)
        return self.A.with_values(m)

    def probe_product(self, Vc, k):
        """U = A V for a column-major probe block Vc (k x n float32, row j = column j)."""
        torch = _torch()
        U = torch.empty_like(Vc)
        _check(lib().spai_probe_product(self.A.c, _ptr(Vc), int(k), _ptr(U), _stream()), "spai_probe_product")
        return U

    def train_step(self, params, m, v, Vc, U, k, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, loss=None):
        """One fused training step (loss/gradient then Adam) via spai_train_step;
        returns the device loss (before the update)."""
        torch = _torch()
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=params.device)
        hyper = (ctypes.c_float * 4)(lr, b1, b2, eps)
        _check(lib().spai_train_step(self.A.c, _ptr(self.feat), _ptr(self.rowidx), _ptr(self.diag), _ptr(Vc),
                                     _ptr(U), k, _ptr(params), _ptr(m), _ptr(v), int(t), hyper, _ptr(loss),
                                     _ptr(self.ws), self.ws.numel(), _stream()), "spai_train_step")
        return loss

    def loss_grad(self, params, Vc, U, k):
        torch = _torch()
        dev = params.device
        m = torch.empty(self.A.nnz, dtype=torch.float32, device=dev)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        grad = torch.empty(NPARAM, dtype=torch.float32, device=dev)
        _check(lib().spai_loss_grad(self.A.c, _ptr(self.feat), _ptr(self.rowidx), _ptr(self.diag), _ptr(params),
                                    _ptr(Vc), _ptr(U), k, _ptr(m), _ptr(loss), _ptr(grad), _ptr(self.ws),
                                    self.ws.numel(), _stream()), "spai_loss_grad")
        return loss, grad


def workspace_bytes(A, k_max: int = 8) -> int:
    return int(lib().spai_workspace_bytes(A.n, A.nnz, k_max))


def adam(params, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(lib().spai_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(t), float(lr), float(b1), float(b2),
                           float(eps), _stream()), "spai_adam")


def init_params(seed: int, device="cuda"):
    """Xavier-uniform hidden layers, zero last layer: the untrained net is Jacobi.
    (The seeded draw is input generation; it matches oracle.spai.init_params.)"""
    torch = _torch()
    import math
    rng = np.random.default_rng(seed)
    th = np.zeros(NPARAM)
    th[:768] = (rng.uniform(-1, 1, (64, 12)) * math.sqrt(6.0 / 76)).ravel()
    th[832:832 + 4096] = (rng.uniform(-1, 1, (64, 64)) * math.sqrt(6.0 / 128)).ravel()
    return torch.from_numpy(th.astype(np.float32)).to(device)


LAYOUT = "W1[64x12] row-major, b1[64], W2[64x64] row-major, b2[64], w3[64], b3 (float32)"


def save_params(path: str, params) -> str:
    """Write trained parameters to an .npz with their layout and the SHA-256 of the
    float32 bytes; returns the digest."""
    import hashlib
    th = np.ascontiguousarray(params.detach().cpu().numpy() if hasattr(params, "detach") else params,
                              dtype=np.float32)
    if th.shape != (NPARAM,):
        raise ValueError(f"expected {NPARAM} parameters")
    digest = hashlib.sha256(th.tobytes()).hexdigest()
    np.savez(path, params=th, layout=np.array(LAYOUT), sha256=np.array(digest))
    return digest


def load_params(path: str, device="cuda"):
    """Read parameters written by save_params; the digest and layout must match."""
    import hashlib
    with np.load(path, allow_pickle=False) as z:
        th = np.ascontiguousarray(z["params"], dtype=np.float32)
        digest, layout = str(z["sha256"]), str(z["layout"])
    if layout != LAYOUT or th.shape != (NPARAM,):
        raise ValueError("parameter file has a different layout")
    if hashlib.sha256(th.tobytes()).hexdigest() != digest:
        raise ValueError("parameter file checksum mismatch")
    return _torch().from_numpy(th).to(device)


def probe_block(A: CSR, b, seed: int, k_rad=4, steps=(1, 4, 16, 64)):
    """V = [Rademacher columns | r_i / ||r_i|| of plain p-BiCGStab at the given iterations]
    as a column-major k x n float32 tensor (row j = column j of V).  The Rademacher
    columns are seeded input draws; the residuals come from the GPU solver (r_out) and are
    normalised and rounded by spai_probe_column."""
    torch = _torch()
    from synthgen import rademacher
    dev = A.val.device
    k = k_rad + len(steps)
    Vc = torch.empty((k, A.n), dtype=torch.float32, device=dev)
    Vc[:k_rad] = torch.from_numpy(np.ascontiguousarray(rademacher(A.n, k_rad, seed).T.astype(np.float32))).to(dev)
    r = torch.empty(A.n, dtype=torch.float64, device=dev)
    ws = _workspace(lib().spai_probe_column_workspace_bytes(A.n), dev)
    for j, s in enumerate(steps):
        sv = Solver(A, tol=0.0, max_iter=int(s))
        sv.solve(b, None, r_out=r)
        _check(lib().spai_probe_column(A.n, _ptr(r), _ptr(Vc[k_rad + j]), _ptr(ws), ws.numel(), _stream()),
               "spai_probe_column")
    return Vc


def train(problems, epochs=30, lr=1e-3, seed=0, device="cuda", log=None):
    """Adam over the training matrices (one step per matrix per epoch, fixed order).

    `problems`: list of synthgen.Problem.  Returns (params, loss history)."""
    torch = _torch()
    params = init_params(seed, device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    data = []
    ws = _workspace(max(workspace_bytes(p.A) for p in problems), device)
    for p in problems:
        A = CSR.from_host(p.A, device)
        sm = SpaiMatrix(A, ws=ws)
        b = torch.from_numpy(p.b).to(device)
        Vc = probe_block(A, b, seed=1000 + int(p.meta.get("seed", 0)))
        U = sm.probe_product(Vc, Vc.shape[0])
        data.append((sm, Vc, U, Vc.shape[0]))
    hist = []
    t = 0
    for ep in range(epochs):
        losses = torch.empty(len(data), dtype=torch.float32, device=device)
        for j, (sm, Vc, U, k) in enumerate(data):
            t += 1
            sm.train_step(params, m, v, Vc, U, k, t, lr=lr, loss=losses[j:j + 1])
        hist.append(float(np.mean(losses.cpu().numpy().astype(np.float64))))   # host-side reporting
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.5e}")
    return params, hist
