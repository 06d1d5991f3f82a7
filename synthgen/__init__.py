"""Seeded synthetic inputs shared by the GPU path, the tests and the oracle.

This module builds problem instances only: CSR matrices, exact solutions x*,
right-hand sides b = A x*, and random probe blocks.  It holds none of the
solver's arithmetic (no Krylov recurrences, no dot-product accumulation); the
single product b = A x* is delegated to scipy's CSR mat-vec so that both sides
receive the same b without either side computing it.

The paper evaluates on SuiteSparse matrices (Section 3, Table 1), which are not
available here; the families below stand in for them:

* ``cd_stencil``  - convection-diffusion, -div(kappa grad u) + v.grad u on the
  unit square / cube, Dirichlet 0, first-order upwind convection, 5-point (2D)
  or 7-point (3D) stencil, rows scaled by h^2;
* ``random_unsym`` - random unsymmetric rows with lognormal lengths, mostly
  banded columns plus a global fraction, strictly diagonally dominant.

Layout: CSR with int32 ``row_ptr[n+1]`` and ``col_idx[nnz]`` (columns ascending
within a row) and float64 ``val[nnz]``.  Node ordering i + N*j (+ N^2*k), with
the x index fastest.

Draw order of every generator (``numpy.random.default_rng(seed)``): the
coefficient field / matrix entries first, then any direction vector, then
x* = uniform(-1, 1, n).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSR", "Problem", "cd_stencil", "random_unsym", "problem", "training_params",
    "rademacher", "CONFIG_NAMES",
]


@dataclasses.dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def diag(self) -> np.ndarray:
        """Diagonal entries (0 where absent); a structural read, no arithmetic."""
        d = np.zeros(self.n)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        m = rows == self.col_idx
        d[rows[m]] = self.val[m]
        return d


@dataclasses.dataclass
class Problem:
    name: str
    A: CSR
    xstar: np.ndarray
    b: np.ndarray
    meta: dict


def _face_coeffs(kap: np.ndarray | None, shape: tuple, axis: int):
    """Diffusion coefficient on the lower and upper face of every cell along ``axis``.

    Constant coefficients give 1 everywhere.  For a cell-wise field kappa the face
    value is the harmonic mean 2 k_P k_nb / (k_P + k_nb) between neighbours and k_P
    on a boundary face.
    """
    if kap is None:
        ones = np.ones(shape)
        return ones, ones
    lo = kap.copy()
    hi = kap.copy()
    sl_a = [slice(None)] * len(shape)
    sl_b = [slice(None)] * len(shape)
    sl_a[axis] = slice(1, None)
    sl_b[axis] = slice(None, -1)
    ka, kb = kap[tuple(sl_a)], kap[tuple(sl_b)]
    harm = 2.0 * ka * kb / (ka + kb)
    lo[tuple(sl_a)] = harm  # face between cell p (index>=1) and p-1
    hi[tuple(sl_b)] = harm  # face between cell p and p+1
    return lo, hi


def cd_stencil(N: int, dim: int, velocity, kappa: np.ndarray | None = None) -> CSR:
    """Upwind convection-diffusion matrix on an N^dim interior grid, h = 1/(N+1).

    Row p (scaled by h^2):
      lower neighbour along axis d:  -(D_lo) - h*max(v_d, 0)
      upper neighbour along axis d:  -(D_hi) - h*max(-v_d, 0)
      diagonal: sum of all 2*dim face coefficients + h * sum_d |v_d|
    Neighbours on the Dirichlet boundary are dropped; their face still counts in
    the diagonal.  nnz = 5n - 4N (2D) or 7n - 6N^2 (3D).
    """
    assert dim in (2, 3)
    v = [float(t) for t in velocity]
    assert len(v) == dim
    h = 1.0 / (N + 1)
    shape = (N,) * dim  # numpy axis 0 is the slowest coordinate
    n = N ** dim
    # numpy axis a <-> physical axis d = dim-1-a (x fastest)
    coeff_lo, coeff_hi = [], []
    for d in range(dim):
        a = dim - 1 - d
        lo, hi = _face_coeffs(kappa, shape, a)
        coeff_lo.append(lo.reshape(n))
        coeff_hi.append(hi.reshape(n))
    coords = np.indices(shape).reshape(dim, n)  # coords[a]
    strides = [N ** d for d in range(dim)]
    diag = np.zeros(n)
    for d in range(dim):
        diag = diag + coeff_lo[d]
        diag = diag + coeff_hi[d]
    conv = 0.0
    for d in range(dim):
        conv = conv + abs(v[d])
    diag = diag + h * conv
    # columns in ascending order: -stride_{dim-1} .. -1, 0, +1 .. +stride_{dim-1}
    slots = []
    for d in reversed(range(dim)):
        a = dim - 1 - d
        exists = coords[a] > 0
        val = -coeff_lo[d] - h * max(v[d], 0.0)
        slots.append((-strides[d], exists, val))
    slots.append((0, np.ones(n, dtype=bool), diag))
    for d in range(dim):
        a = dim - 1 - d
        exists = coords[a] < N - 1
        val = -coeff_hi[d] - h * max(-v[d], 0.0)
        slots.append((strides[d], exists, val))
    S = len(slots)
    ex = np.stack([s[1] for s in slots], axis=1)           # [n, S]
    cols = np.arange(n)[:, None] + np.array([s[0] for s in slots])[None, :]
    vals = np.stack([np.broadcast_to(s[2], (n,)) for s in slots], axis=1)
    counts = ex.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[ex].astype(np.int32)
    val = vals[ex].astype(np.float64)
    assert row_ptr[-1] < 2 ** 31
    del S
    return CSR(n, row_ptr.astype(np.int32), col_idx, np.ascontiguousarray(val))


def random_unsym(n: int, rng: np.random.Generator, mu=math.log(14.0), sigma=0.6,
                 kmin=2, kmax=400, band=5000, p_band=0.8, dominance=1.2) -> CSR:
    """Random unsymmetric sparse matrix.

    Off-diagonal count per row k_i = clip(rint(lognormal(mu, sigma)), kmin, kmax).
    Each off-diagonal column is drawn with probability p_band uniformly from
    i + {-band..band} \\ {0}, otherwise uniformly from [0, n); out-of-range columns,
    duplicates and the diagonal are rejected and redrawn.  Values ~ N(0, 1).
    Diagonal = RN(dominance * sum |offdiag|) (math.fsum per row), positive.
    """
    k = np.clip(np.rint(rng.lognormal(mu, sigma, n)), kmin, min(kmax, n - 1)).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    m = rows.shape[0]
    cols = np.full(m, -1, dtype=np.int64)
    pending = np.arange(m)
    while pending.size:
        r = rows[pending]
        near = rng.random(pending.size) < p_band
        off = rng.integers(-band, band, size=pending.size, endpoint=True)
        glob = rng.integers(0, n, size=pending.size)
        c = np.where(near, r + off, glob)
        cols[pending] = c
        # reject out of range, diagonal, duplicates within the row (keep first occurrence)
        bad = (cols < 0) | (cols >= n) | (cols == rows)
        key = rows * n + np.where(bad, -1, cols)
        order = np.lexsort((np.arange(m), key))
        ks = key[order]
        dup = np.zeros(m, dtype=bool)
        dup[order[1:]] = ks[1:] == ks[:-1]
        bad |= dup
        pending = np.nonzero(bad)[0]
    vals = rng.standard_normal(m)
    # sort columns within rows and insert the diagonal
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    absv = np.abs(vals)
    row_start = np.concatenate([[0], np.cumsum(k)])
    diag = np.empty(n)
    for i in range(n):  # fsum: exactly rounded row sums of |offdiag|
        diag[i] = dominance * math.fsum(absv[row_start[i]:row_start[i + 1]])
    all_rows = np.concatenate([rows, np.arange(n)])
    all_cols = np.concatenate([cols, np.arange(n)])
    all_vals = np.concatenate([vals, diag])
    order = np.lexsort((all_cols, all_rows))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k + 1, out=row_ptr[1:])
    assert row_ptr[-1] < 2 ** 31
    return CSR(n, row_ptr.astype(np.int32), all_cols[order].astype(np.int32),
               np.ascontiguousarray(all_vals[order]))


def _rhs(A: CSR, xstar: np.ndarray) -> np.ndarray:
    return np.asarray(A.to_scipy() @ xstar, dtype=np.float64)


def _unit_dir(rng, dim):
    d = rng.standard_normal(dim)
    return d / np.linalg.norm(d)


CONFIG_NAMES = ("cd2d_64", "cd3d_128", "rand_1m", "cd3d_256_var", "spai_eval_128")


def problem(name: str, scale: int | None = None) -> Problem:
    """Named workloads.  ``scale`` overrides the grid size N (or n for the random
    family) to build a smaller instance of the same family for tests.

    cd2d_64        2D, 64^2, v = (20, 10), D = 1, seed 0
    cd3d_128       3D, 128^3, v = (30, 20, 10), D = 1, seed 1
    rand_1m        random unsymmetric, n = 10^6, seed 2
    cd3d_256_var   3D, 256^3, kappa = exp(N(0,1)) per cell, v = (50, 25, 10), seed 3
    spai_eval_128  3D, 128^3, kappa = exp(N(0,1)), |v| = Peclet 50, direction from seed 4
    """
    if name == "cd2d_64":
        N = scale or 64
        rng = np.random.default_rng(0)
        A = cd_stencil(N, 2, (20.0, 10.0))
        meta = dict(N=N, dim=2, velocity=(20.0, 10.0), seed=0)
    elif name == "cd3d_128":
        N = scale or 128
        rng = np.random.default_rng(1)
        A = cd_stencil(N, 3, (30.0, 20.0, 10.0))
        meta = dict(N=N, dim=3, velocity=(30.0, 20.0, 10.0), seed=1)
    elif name == "rand_1m":
        n = scale or 1_000_000
        rng = np.random.default_rng(2)
        A = random_unsym(n, rng)
        meta = dict(n=n, seed=2)
    elif name == "cd3d_256_var":
        N = scale or 256
        rng = np.random.default_rng(3)
        kap = np.exp(rng.standard_normal((N, N, N)))
        A = cd_stencil(N, 3, (50.0, 25.0, 10.0), kap)
        meta = dict(N=N, dim=3, velocity=(50.0, 25.0, 10.0), seed=3, kappa="exp(N(0,1))")
    elif name == "spai_eval_128":
        N = scale or 128
        rng = np.random.default_rng(4)
        kap = np.exp(rng.standard_normal((N, N, N)))
        vel = tuple(50.0 * _unit_dir(rng, 3))
        A = cd_stencil(N, 3, vel, kap)
        meta = dict(N=N, dim=3, velocity=vel, seed=4, peclet=50.0, kappa="exp(N(0,1))")
    else:
        raise KeyError(name)
    xstar = rng.uniform(-1.0, 1.0, A.n)
    return Problem(name, A, xstar, _rhs(A, xstar), meta)


def training_params(seed: int) -> dict:
    """Parameters of one learned-preconditioner training matrix (seeds 100..299).

    dim in {2, 3} with p = 1/2; n log-uniform on [16384, 262144] -> N = round(n^(1/dim));
    Peclet log-uniform on [1, 100]; direction uniform on the sphere; v = Pe * dir.
    The kappa field exp(N(0,1)) per cell is drawn by ``training_problem``.
    """
    rng = np.random.default_rng(seed)
    dim = 2 if rng.random() < 0.5 else 3
    n_target = math.exp(rng.uniform(math.log(16384), math.log(262144)))
    N = int(round(n_target ** (1.0 / dim)))
    pe = math.exp(rng.uniform(0.0, math.log(100.0)))
    vel = tuple(pe * _unit_dir(rng, dim))
    return dict(seed=seed, dim=dim, N=N, peclet=pe, velocity=vel)


def training_problem(seed: int, N: int | None = None) -> Problem:
    p = training_params(seed)
    if N is not None:
        p["N"] = N
    rng = np.random.default_rng(10_000 + seed)
    kap = np.exp(rng.standard_normal((p["N"],) * p["dim"]))
    A = cd_stencil(p["N"], p["dim"], p["velocity"], kap)
    xstar = rng.uniform(-1.0, 1.0, A.n)
    return Problem(f"train_{seed}", A, xstar, _rhs(A, xstar), p)


def save_problem(path: str, prob: Problem) -> str:
    """Cache a generated problem as .npz with the SHA-256 of its arrays; returns it."""
    import hashlib
    import json
    arrays = {"row_ptr": prob.A.row_ptr, "col_idx": prob.A.col_idx, "val": prob.A.val,
              "xstar": prob.xstar, "b": prob.b}
    h = hashlib.sha256()
    for k in sorted(arrays):
        h.update(np.ascontiguousarray(arrays[k]).tobytes())
    digest = h.hexdigest()
    meta = json.dumps({"name": prob.name, "n": prob.A.n, "meta": prob.meta}, default=float)
    np.savez(path, **arrays, meta=np.array(meta), sha256=np.array(digest))
    return digest


def load_problem(path: str) -> Problem:
    """Load a problem written by save_problem, verifying its checksum."""
    import hashlib
    import json
    with np.load(path, allow_pickle=False) as z:
        arrays = {k: z[k] for k in ("row_ptr", "col_idx", "val", "xstar", "b")}
        digest, meta = str(z["sha256"]), json.loads(str(z["meta"]))
    h = hashlib.sha256()
    for k in sorted(arrays):
        h.update(np.ascontiguousarray(arrays[k]).tobytes())
    if h.hexdigest() != digest:
        raise ValueError(f"{path}: checksum mismatch")
    A = CSR(int(meta["n"]), arrays["row_ptr"], arrays["col_idx"], arrays["val"])
    return Problem(meta["name"], A, arrays["xstar"], arrays["b"], meta["meta"])


def rademacher(n: int, k: int, seed: int) -> np.ndarray:
    """n x k column-major (Fortran order) block of +-1 probes."""
    rng = np.random.default_rng(seed)
    v = rng.integers(0, 2, size=(k, n)).astype(np.float64) * 2.0 - 1.0
    return np.asfortranarray(v.T)


def uniform_vec(n: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def cancelling_vec(n: int, seed: int, big_exp=300, n_small=16) -> np.ndarray:
    """Ill-conditioned dot input against y = 1: pairs (u, -u) with exponents up to
    big_exp cancel exactly, so the exact sum is that of n_small values in [-1, 1];
    condition number sum|x| / |sum x| is astronomically large.  Seeded shuffle."""
    rng = np.random.default_rng(seed)
    h = (n - n_small) // 2
    u = np.ldexp(rng.uniform(1.0, 2.0, h), rng.integers(-big_exp, big_exp, size=h, endpoint=True))
    small = rng.uniform(-1.0, 1.0, n - 2 * h)
    return rng.permutation(np.concatenate([u, -u, small]))


def wide_exponent_vec(n: int, seed: int, emin=-1000, emax=1000) -> np.ndarray:
    """Signed doubles with uniformly random exponents in [emin, emax]."""
    rng = np.random.default_rng(seed)
    m = rng.uniform(1.0, 2.0, n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    e = rng.integers(emin, emax, size=n, endpoint=True)
    return np.ldexp(m, e)
