"""Pins of the learned-preconditioner oracle.

Central finite differences of the loss in float64 pin the whole analytic gradient
chain (SDDMM, skip connection, both GELU layers, biases); the untrained net (zero
last layer) is exactly Jacobi; the features are invariant under A -> cA and the
m values scale as 1/c; the bf16 rounding matches its definition on hand-picked
values; Adam matches its closed form on the first step (lr * sign(g)); all twelve
features of a hand-worked unsymmetric 4 x 4 matrix are written out and must match.
"""
import math

import numpy as np
import pytest

import synthgen as g
from oracle import spai


@pytest.fixture(scope="module")
def small():
    p = g.problem("spai_eval_128", scale=5)
    V = g.rademacher(p.A.n, 3, 7) * 0.5 + np.random.default_rng(0).standard_normal((p.A.n, 3)) * 0.1
    return p.A, np.asfortranarray(V)


def test_param_count():
    assert spai.NPARAM == 5057


def test_untrained_is_jacobi(small):
    A, _ = small
    th = spai.init_params(0)
    m = spai.m_values(A, th)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    expect = np.where(rows == A.col_idx, 1.0 / A.diag()[rows], 0.0)
    assert np.allclose(m, expect, rtol=0, atol=0)


def test_features_scale_invariant(small):
    A, _ = small
    phi = spai.features(A)
    A3 = g.CSR(A.n, A.row_ptr, A.col_idx, A.val * 3.0)
    assert np.allclose(spai.features(A3), phi, rtol=1e-14, atol=1e-15)
    th = spai.init_params(1)
    th[-65:-1] = np.random.default_rng(2).standard_normal(64) * 0.1
    assert np.allclose(spai.m_values(A3, th) * 3.0, spai.m_values(A, th), rtol=1e-13)


def test_features_closed_form_entries():
    A = g.cd_stencil(4, 2, (0.0, 0.0))  # symmetric Laplacian: diag 4, off -1
    phi = spai.features(A)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = rows != A.col_idx
    assert np.allclose(phi[off, 0], -0.25) and np.allclose(phi[off, 1], -0.25)
    assert np.allclose(phi[:, 2], 1.0) and np.allclose(phi[:, 3], 1.0)
    assert np.allclose(phi[off, 11], 0.0)  # symmetric: zero local Peclet number
    assert np.allclose(phi[~off, 10], 1.0) and np.allclose(phi[off, 10], 0.0)


# A hand-worked unsymmetric 4 x 4 matrix (negative diagonal in row 2, a missing transpose
# entry at (1, 2)) and all twelve features of its eleven entries, worked out by hand:
#   row abs sums R = (7, 7, 12, 4), column abs sums C = (7, 7, 9, 7),
#   row lengths (3, 2, 3, 3) (max 3), max |j - i| per row (3, 1, 1, 3).
HAND_A = [(0, 0, 4.0), (0, 1, -1.0), (0, 3, 2.0),
          (1, 0, -2.0), (1, 1, 5.0),
          (2, 1, 1.0), (2, 2, -8.0), (2, 3, 3.0),
          (3, 0, 1.0), (3, 2, -1.0), (3, 3, 2.0)]
F = __import__("fractions").Fraction
HAND_PHI = [
    # a_ij/|aii| a_ji/|aii| a_jj/|aii| sgn  R_i/|aii| R_j/|ajj| C_i/|aii| C_j/|ajj| len   (j-i)/mo [i=j] Pe
    [1,        1,        1,        1,  F(7, 4), F(7, 4), F(7, 4), F(7, 4), 1,       0,       1, 0],        # (0,0)
    [F(-1, 4), F(-1, 2), F(5, 4),  1,  F(7, 4), F(7, 5), F(7, 4), F(7, 5), 1,       F(1, 3), 0, F(1, 3)],  # (0,1)
    [F(1, 2),  F(1, 4),  F(1, 2),  1,  F(7, 4), 2,       F(7, 4), F(7, 2), 1,       1,       0, F(1, 3)],  # (0,3)
    [F(-2, 5), F(-1, 5), F(4, 5),  1,  F(7, 5), F(7, 4), F(7, 5), F(7, 4), F(2, 3), -1,      0, F(1, 3)],  # (1,0)
    [1,        1,        1,        1,  F(7, 5), F(7, 5), F(7, 5), F(7, 5), F(2, 3), 0,       1, 0],        # (1,1)
    [F(1, 8),  0,        F(5, 8),  -1, F(3, 2), F(7, 5), F(9, 8), F(7, 5), 1,       -1,      0, 1],        # (2,1)
    [-1,       -1,       -1,       -1, F(3, 2), F(3, 2), F(9, 8), F(9, 8), 1,       0,       1, 0],        # (2,2)
    [F(3, 8),  F(-1, 8), F(1, 4),  -1, F(3, 2), 2,       F(9, 8), F(7, 2), 1,       1,       0, 2],        # (2,3)
    [F(1, 2),  1,        2,        1,  2,       F(7, 4), F(7, 2), F(7, 4), 1,       -1,      0, F(1, 3)],  # (3,0)
    [F(-1, 2), F(3, 2),  -4,       1,  2,       F(3, 2), F(7, 2), F(9, 8), 1,       F(-1, 3), 0, 2],       # (3,2)
    [1,        1,        1,        1,  2,       2,       F(7, 2), F(7, 2), 1,       0,       1, 0],        # (3,3)
]


def test_features_hand_worked_unsymmetric():
    rows = [i for i, _, _ in HAND_A]
    rp = np.zeros(5, dtype=np.int32)
    np.add.at(rp, np.array(rows) + 1, 1)
    A = g.CSR(4, np.cumsum(rp).astype(np.int32), np.array([j for _, j, _ in HAND_A], dtype=np.int32),
              np.array([v for _, _, v in HAND_A]))
    phi = spai.features(A)
    expect = np.array([[float(v) for v in row] for row in HAND_PHI])
    assert phi.shape == expect.shape
    # every value is a ratio of small integers: float64 division rounds it once
    assert np.array_equal(phi, expect), np.argwhere(phi != expect)


def test_gradient_matches_finite_differences(small):
    A, V = small
    rng = np.random.default_rng(3)
    th = spai.init_params(4)
    th += rng.standard_normal(th.size) * 0.05
    L, grad = spai.loss_and_grad(A, th, V)
    idx = np.concatenate([rng.choice(768, 6, replace=False),                    # W1
                          768 + rng.choice(64, 3, replace=False),              # b1
                          832 + rng.choice(4096, 6, replace=False),            # W2
                          4928 + rng.choice(64, 3, replace=False),             # b2
                          4992 + rng.choice(64, 4, replace=False), [5056]])    # w3, b3
    for k in idx:
        h = 1e-6 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (spai.loss_and_grad(A, tp, V)[0] - spai.loss_and_grad(A, tm, V)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1e-8, abs(grad).max()), (k, fd, grad[k])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 1e-30], dtype=np.float32)
    out = spai.to_bf16(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                     # tie -> even (mantissa ...0)
    assert out[2] == 1.0 + 2 ** -7           # exactly representable
    assert out[3] == 1.0 + 2 ** -6           # tie -> even (mantissa ...10)
    assert out[4] == -2.5
    assert abs(out[5] - 1e-30) <= 1e-30 * 2 ** -8


def test_adam_first_step_is_signed_lr():
    g0 = np.array([0.3, -2.0, 1e-3])
    th, m, v = spai.adam_step(np.zeros(3), g0, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g0))


def test_training_reduces_loss(small):
    A, V = small
    th = spai.init_params(5)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = spai.loss_and_grad(A, th, V)[0]
    for t in range(1, 41):
        L, gr = spai.loss_and_grad(A, th, V)
        th, m, v = spai.adam_step(th, gr, m, v, t, lr=3e-3)
    assert spai.loss_and_grad(A, th, V)[0] < 0.9 * L0


def test_probe_block_hand_worked():
    """A = diag(1, 2), b = (1, 1): the first p-BiCGStab iteration gives alpha = 2/3,
    q = (1/3, -1/3), y = A q, omega = (q, y)/(y, y) = 3/5 and r_1 = q - omega y =
    (2/15, 1/15), so the residual probe column is (2, 1)/sqrt(5); the Rademacher
    columns hold +-1 only."""
    A = g.CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 2.0]))
    V = spai.probe_block(A, np.array([1.0, 1.0]), seed=3, k_rad=2, steps=(1,))
    assert V.shape == (2, 3)
    assert set(np.unique(V[:, :2]).tolist()) <= {-1.0, 1.0}
    expect = np.array([2.0, 1.0]) / math.sqrt(5.0)
    assert np.allclose(V[:, 2], expect, rtol=8 * 2.0 ** -53, atol=0)   # a few roundings
