"""Fused p-BiCGStab phase kernels vs the oracle's literal-order updates.

Given identical inputs and scalars, every updated vector must be bit-identical to
the paper's recurrences (Algorithm 2, the p/s/z/q/y and x/r/w updates) evaluated with
separately rounded operations, and the fused dot products must be bit-identical to
the oracle's exact dots of the updated vectors.
"""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
from oracle import ctier
from tests.gpu_util import same_bits, to_dev

pytestmark = pytest.mark.gpu


def rand_vecs(n, seed):
    rng = np.random.default_rng(seed)
    names = ("x", "r", "rhat", "w", "t", "p", "s", "z", "q", "y", "v")
    V = {k: rng.standard_normal(n) * 10.0 ** rng.integers(-3, 3) for k in names}
    V["v"][::5] *= 1e-180  # wide exponent range inside the vectors
    return V


@pytest.mark.parametrize("n", [1, 100, 4096, 300007])
@pytest.mark.parametrize("first", [False, True])
def test_phase_a(n, first):
    V = rand_vecs(n, n)
    alpha, beta, omega = 0.7311, -1.25e-3, 3.5
    # oracle: literal order (numpy rounds every operation)
    r, w, t, v, rh = V["r"], V["w"], V["t"], V["v"], V["rhat"]
    if first:
        p, s, z = r.copy(), w.copy(), t.copy()
    else:
        p = r + beta * (V["p"] - omega * V["s"])
        s = w + beta * (V["s"] - omega * V["z"])
        z = t + beta * (V["z"] - omega * v)
    q = r - alpha * s
    y = w - alpha * z
    TV = {k: to_dev(a) for k, a in V.items()}
    scal = to_dev(np.array([alpha, beta, omega]))
    dots = pk.pbcg_phase_a(TV, scal, first).cpu().numpy()
    for name, ref in (("p", p), ("s", s), ("z", z), ("q", q), ("y", y)):
        assert np.array_equal(TV[name].cpu().numpy().view(np.uint64), ref.view(np.uint64)), name
    expect = [ctier.exact_dot(q, y), ctier.exact_dot(y, y), ctier.exact_dot(rh, s), ctier.exact_dot(rh, z)]
    for a, b in zip(dots, expect):
        assert same_bits(a, b)


@pytest.mark.parametrize("n", [1, 100, 4096, 300007])
def test_phase_b(n):
    V = rand_vecs(n, n + 1)
    alpha, omega = -0.21, 1.9e-2
    x = (V["x"] + alpha * V["p"]) + omega * V["q"]
    r = V["q"] - omega * V["y"]
    w = V["y"] - omega * (V["t"] - alpha * V["v"])
    TV = {k: to_dev(a) for k, a in V.items()}
    scal = to_dev(np.array([alpha, 123.0, omega]))
    dots = pk.pbcg_phase_b(TV, scal).cpu().numpy()
    for name, ref in (("x", x), ("r", r), ("w", w)):
        assert np.array_equal(TV[name].cpu().numpy().view(np.uint64), ref.view(np.uint64)), name
    rh = V["rhat"]
    expect = [ctier.exact_dot(rh, r), ctier.exact_dot(rh, w), ctier.exact_dot(r, r)]
    for a, b in zip(dots, expect):
        assert same_bits(a, b)


def test_phase_a_full_size():
    """2^24 rows (the 256^3 workload's vector length): updated vectors bit for bit against
    the literal-order recurrences, dots against the oracle's exact dots of those vectors."""
    n = 1 << 24
    V = rand_vecs(n, 7)
    alpha, beta, omega = 0.5, 0.25, -2.0
    s = V["w"] + beta * (V["s"] - omega * V["z"])
    z = V["t"] + beta * (V["z"] - omega * V["v"])
    q = V["r"] - alpha * s
    y = V["w"] - alpha * z
    TV = {k: to_dev(a) for k, a in V.items()}
    scal = to_dev(np.array([alpha, beta, omega]))
    dots = pk.pbcg_phase_a(TV, scal, False).cpu().numpy()
    torch.cuda.synchronize()
    for name, ref in (("s", s), ("z", z), ("q", q), ("y", y)):
        assert np.array_equal(TV[name].cpu().numpy().view(np.uint64), ref.view(np.uint64)), name
    expect = [ctier.exact_dot(q, y), ctier.exact_dot(y, y), ctier.exact_dot(V["rhat"], s),
              ctier.exact_dot(V["rhat"], z)]
    for a, b in zip(dots, expect):
        assert same_bits(a, b)
