"""Learned sparse approximate inverse (SPAI) -- oracle, float64 unless stated.

The paper mentions preconditioned variants only (Section 2, the residual replacement
paragraph: r̄ = M⁻¹ r); the learned preconditioner follows the build's own definition:
M has A's sparsity pattern and its value at (i, j) is

    m_ij = ([i = j] + f_theta(phi_ij)) / a_ii

where f_theta is an MLP 12 -> 64 -> 64 -> 1 with GELU (erf form) and phi_ij are 12
per-nonzero features (below).  With the last layer zero the network is exactly Jacobi.
Training minimises L = ||M A V - V||_F^2 / (k n) over probe blocks V (n x k).

Features phi_ij (scale invariant under A -> cA, c > 0):
  0 a_ij/|a_ii|          1 a_ji/|a_ii| (0 if absent)   2 a_jj/|a_ii|      3 sign(a_ii)
  4 R_i/|a_ii|           5 R_j/|a_jj|                  6 C_i/|a_ii|       7 C_j/|a_jj|
  8 len_i / max_len      9 (j-i)/max_{k in row i}|k-i| (0 if that max is 0)
 10 [i = j]             11 |a_ij - a_ji| / max(|a_ij + a_ji|, 2^-126) (0 on the diagonal)
R = row sums of |a|, C = column sums of |a|, len = entries per row.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np

NF, H = 12, 64
NPARAM = H * NF + H + H * H + H + H + 1  # 5057
TINY = 2.0 ** -126


# ------------------------------------------------------------------ features
def features(A) -> np.ndarray:
    n = A.n
    rp = A.row_ptr.astype(np.int64)
    ci = A.col_idx.astype(np.int64)
    a = A.val.astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    diag = np.zeros(n)
    dmask = rows == ci
    diag[rows[dmask]] = a[dmask]
    absd = np.abs(diag)
    R = np.bincount(rows, weights=np.abs(a), minlength=n)
    C = np.bincount(ci, weights=np.abs(a), minlength=n)
    lens = np.diff(rp).astype(np.float64)
    maxlen = lens.max() if n else 1.0
    off = np.abs(ci - rows).astype(np.float64)
    maxoff = np.zeros(n)
    np.maximum.at(maxoff, rows, off)
    # a_ji by lookup in row j
    key = rows * n + ci
    order = np.argsort(key)
    skey = key[order]
    tkey = ci * n + rows
    pos = np.searchsorted(skey, tkey)
    pos = np.minimum(pos, len(skey) - 1)
    found = skey[pos] == tkey
    aji = np.where(found, a[order[pos]], 0.0)
    phi = np.zeros((len(a), NF))
    phi[:, 0] = a / absd[rows]
    phi[:, 1] = aji / absd[rows]
    phi[:, 2] = diag[ci] / absd[rows]
    phi[:, 3] = np.sign(diag[rows])
    phi[:, 4] = R[rows] / absd[rows]
    phi[:, 5] = R[ci] / absd[ci]
    phi[:, 6] = C[rows] / absd[rows]
    phi[:, 7] = C[ci] / absd[ci]
    phi[:, 8] = lens[rows] / maxlen
    mo = maxoff[rows]
    phi[:, 9] = np.where(mo > 0, (ci - rows) / np.where(mo > 0, mo, 1.0), 0.0)
    phi[:, 10] = dmask.astype(np.float64)
    pe = np.abs(a - aji) / np.maximum(np.abs(a + aji), TINY)
    phi[:, 11] = np.where(dmask, 0.0, pe)
    return phi


# ------------------------------------------------------------------ parameters
def unpack(theta):
    """Flat layout: W1[64x12] row-major, b1[64], W2[64x64] row-major, b2[64], w3[64], b3."""
    t = np.asarray(theta)
    o = 0
    W1 = t[o:o + H * NF].reshape(H, NF); o += H * NF
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + H * H].reshape(H, H); o += H * H
    b2 = t[o:o + H]; o += H
    w3 = t[o:o + H]; o += H
    b3 = t[o]
    return W1, b1, W2, b2, w3, b3


def init_params(seed: int) -> np.ndarray:
    """Xavier-uniform hidden layers, zero last layer (the untrained net is Jacobi)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NPARAM)
    W1, b1, W2, b2, w3, b3 = unpack(th)
    W1[:] = rng.uniform(-1, 1, (H, NF)) * math.sqrt(6.0 / (NF + H))
    W2[:] = rng.uniform(-1, 1, (H, H)) * math.sqrt(6.0 / (H + H))
    return th


# ------------------------------------------------------------------ MLP
_erf = np.vectorize(math.erf)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(theta, phi):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    z1 = phi @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    f = h2 @ w3 + b3
    return f, (z1, h1, z2, h2)


def m_values(A, theta, phi=None):
    phi = features(A) if phi is None else phi
    f, _ = forward(theta, phi)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    dg = A.diag()
    return (phi[:, 10] + f) / dg[rows]


def spmm(A, vals, X):
    """Y = A_vals X (X: n x k), rows summed left to right (float64)."""
    rp = A.row_ptr.astype(np.int64)
    lens = np.diff(rp)
    Y = np.zeros((A.n, X.shape[1]))
    for k in range(int(lens.max()) if A.n else 0):
        rows = np.nonzero(lens > k)[0]
        idx = rp[rows] + k
        Y[rows] = Y[rows] + vals[idx][:, None] * X[A.col_idx[idx]]
    return Y


def loss_and_grad(A, theta, V, phi=None):
    """L = ||M U - V||_F^2 / (k n) with U = A V; returns (L, dL/dtheta)."""
    phi = features(A) if phi is None else phi
    n, k = V.shape
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr.astype(np.int64)))
    cols = A.col_idx.astype(np.int64)
    dg = A.diag()
    U = spmm(A, A.val, V)
    f, (z1, h1, z2, h2) = forward(theta, phi)
    m = (phi[:, 10] + f) / dg[rows]
    R = spmm(A, m, U) - V
    L = float(np.sum(R * R)) / (k * n)
    g_m = (2.0 / (k * n)) * np.sum(R[rows] * U[cols], axis=1)   # dL/dm_ij (SDDMM)
    g_f = g_m / dg[rows]                                           # dL/df_ij
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    grad = np.zeros(NPARAM)
    G1, gb1, G2, gb2, gw3, _ = unpack(grad)
    gw3[:] = g_f @ h2
    grad[-1] = g_f.sum()
    dz2 = (g_f[:, None] * w3[None, :]) * gelu_grad(z2)
    G2[:] = dz2.T @ h1
    gb2[:] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    G1[:] = dz1.T @ phi
    gb1[:] = dz1.sum(axis=0)
    return L, grad


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), t >= 1; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ bf16 inference emulation
def to_bf16(x):
    """Round float32 values to bfloat16 (nearest-even), returned as float32."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), x, out)


def infer_bf16(A, theta, phi=None):
    """Weights and layer inputs rounded to bf16, products accumulated in float64 here
    (the GPU accumulates in float32 in its own order), GELU on the accumulated values."""
    phi = features(A) if phi is None else phi
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    return infer_bf16_values(theta, phi, A.diag()[rows])


def infer_bf16_values(theta, phi, a_ii):
    """The bf16 inference of ``infer_bf16`` for given feature rows phi (k x 12) and the
    diagonal entry a_ii of each one's row (any subset of the nonzeros)."""
    W1, b1, W2, b2, w3, b3 = [np.asarray(t, dtype=np.float32) for t in unpack(theta)]
    x0 = to_bf16(phi.astype(np.float32)).astype(np.float64)
    z1 = x0 @ to_bf16(W1).astype(np.float64).T + b1
    h1 = to_bf16(gelu(z1).astype(np.float32)).astype(np.float64)
    z2 = h1 @ to_bf16(W2).astype(np.float64).T + b2
    h2 = to_bf16(gelu(z2).astype(np.float32)).astype(np.float64)
    f = h2 @ to_bf16(w3).astype(np.float64) + float(b3)
    return (phi[:, 10] + f) / a_ii


# ------------------------------------------------------------------ probe blocks
def _exact_dot(a, b):
    from . import exact
    if a.size <= 20000:
        return exact.exact_dot(a.tolist(), b.tolist())
    from . import ctier
    return ctier.exact_dot(a, b)


def probe_block(A, b, seed, dot=None, k_rad=4, steps=(1, 4, 16, 64)):
    """V = [k_rad Rademacher columns | normalised residuals r_i / ||r_i|| of a plain
    p-BiCGStab run on (A, b) at the iterations in `steps` (or the last available)].
    ||r|| is the square root of the exact (r, r), rounded once -- the norm every inner
    product of the method uses; a zero residual gives a zero column."""
    from synthgen import rademacher
    from . import solvers
    n = A.n
    cols = [rademacher(n, k_rad, seed)]
    res = solvers.pbicgstab(A, b, tol=0.0, max_iter=max(steps), record=max(steps), dot=dot)
    for s in steps:
        it = res.iterates[min(s, len(res.iterates)) - 1] if res.iterates else None
        r = it[1] if it is not None else b
        nrm = math.sqrt(_exact_dot(r, r))
        cols.append((r / nrm if nrm > 0 else np.zeros(n))[:, None])
    return np.asfortranarray(np.concatenate(cols, axis=1))
