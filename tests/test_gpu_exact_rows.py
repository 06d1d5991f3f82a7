"""Exactly rounded SpMV rows (csr_spmv_exact; solver option exact_rows) against the
oracle's definition: every row one exact sum, rounded once -- bit for bit, on ragged,
empty, long, cancelling, wide-exponent and non-finite rows, on FP32 values, and on
sampled rows of the full-size workloads; solves with exact rows bit for bit against the
oracle's solve with the same definition."""
import numpy as np
import pytest
import torch

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import solvers
from oracle.spmv import resid_exact, spmv_exact
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def same(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nan = np.isnan(a) & np.isnan(b)
    return np.array_equal(bits(np.where(nan, 0.0, a)), bits(np.where(nan, 0.0, b)))


def csr_rows(rows, n):
    rp, ci, va = [0], [], []
    for r in rows:
        for c, v in r:
            ci.append(c)
            va.append(v)
        rp.append(len(ci))
    return g.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va, dtype=np.float64))


def cases():
    rng = np.random.default_rng(3)
    out = []
    n = 700
    rows = []
    for i in range(n):
        k = int(rng.integers(0, 40)) if i % 50 else 0           # empty rows, up to 39 entries
        cols = np.sort(rng.choice(n, size=k, replace=False))
        vals = rng.standard_normal(k) * np.exp2(rng.integers(-60, 60, k))
        rows.append(list(zip(cols.tolist(), vals.tolist())))
    rows[7] = [(c, 1e16 if c % 2 else -1e16) for c in range(0, 600, 3)] + [(699, 0.5)]   # cancelling, 201 entries
    out.append(("mixed_700", csr_rows(rows, n), rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))))
    # products beyond DBL_MAX and below the subnormal range, exactly cancelling
    big, tiny = 2.0 ** 600, 2.0 ** -600
    rows = [[(0, big), (1, -big), (2, 1.0)], [(0, tiny), (1, tiny)], [(0, 3.0), (1, 2.0 ** -1074)]]
    out.append(("extremes", csr_rows(rows, 3), np.array([2.0 ** 500, 2.0 ** 500, 2.0 ** -500])))
    # one row of 1500 entries
    rows = [[(c, float(c % 7) - 3.0) for c in range(1500)]] + [[] for _ in range(1499)]
    out.append(("long_row", csr_rows(rows, 1500), rng.uniform(-1, 1, 1500)))
    out.append(("rand_3000", g.problem("rand_1m", scale=3000).A, rng.uniform(-1, 1, 3000)))
    A, x, _ = paths_case()
    out.append(("paths_1400", A, x))
    # long rows: 8 and 16 lanes per row on the register path (mean length 40 and 80)
    for n, lo, hi in ((500, 20, 61), (400, 40, 121)):
        rows = []
        for i in range(n):
            k = int(rng.integers(lo, hi))
            cols = np.sort(rng.choice(n, size=k, replace=False))
            e = rng.integers(-20, 20, k) if i % 5 else rng.integers(-200, 200, k)
            rows.append(list(zip(cols.tolist(), (rng.standard_normal(k) * np.exp2(e)).tolist())))
        out.append((f"long_rows_{n}", csr_rows(rows, n), rng.uniform(-1, 1, n)))
    return out


def paths_case():
    """Rows in blocks of 256 that exercise both row paths of the kernel: rows whose terms
    span a few 32-bit chunks (summed by one lane in registers) and rows spanning more
    (summed by 16 lanes in LDS): a block of narrow rows, a block of only wide rows, blocks
    mixing the two with exact ties, cancellations and subnormal products, and a ragged
    tail.  Returns (A, x, b), all finite."""
    rng = np.random.default_rng(11)
    n = 1400
    x = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-20, 20, n))
    x[900:1000] = rng.choice([1.0, -1.0, 0.5, 2.0 ** -53, 3.0], 100)
    x[1000:1100] = rng.uniform(-1, 1, 100) * 2.0 ** -540
    rows = []
    for i in range(n):
        k = int(rng.integers(0, 24))
        cols = np.sort(rng.choice(n, size=k, replace=False))
        blk = i // 256
        if blk == 1 or (blk in (2, 4) and i % 3 == 0):              # wide: 2^-90 .. 2^90
            vals = rng.standard_normal(k) * np.exp2(rng.integers(-90, 90, k))
        elif blk == 3:                                               # ties and cancellation
            cols = np.sort(rng.choice(np.arange(900, 1000), size=min(k, 100), replace=False))
            vals = rng.choice([1.0, -1.0, 2.0 ** 52, -(2.0 ** 52), 0.5], len(cols))
        elif blk == 4 and i % 3 == 1:                                # subnormal products
            cols = np.sort(rng.choice(np.arange(1000, 1100), size=min(k, 100), replace=False))
            vals = rng.standard_normal(len(cols)) * 2.0 ** -540
        else:
            vals = rng.standard_normal(k)
        rows.append(list(zip(cols.tolist(), vals.tolist())))
    A = csr_rows(rows, n)
    b = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-40, 40, n))
    b[768:1024] = rng.choice([0.0, 1.0, -2.0 ** -53, 2.0 ** 53], 256)
    return A, x, b


@pytest.mark.parametrize("name,A,x", cases(), ids=[c[0] for c in cases()])
def test_exact_rows_bitwise(name, A, x):
    y = pk.csr_spmv_exact(pk.CSR.from_host(A), to_dev(x)).cpu().numpy()
    assert same(y, spmv_exact(A, x))
    # FP32 values: their products are exact in double too
    A32 = g.CSR(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32).astype(np.float64))
    y32 = pk.csr_spmv_exact(pk.CSR.from_host(A, dtype=torch.float32), to_dev(x)).cpu().numpy()
    assert same(y32, spmv_exact(A32, x))


def test_exact_rows_nonfinite():
    """Non-finite products follow the exact dot: NaN, inf * 0, or both infinities -> NaN;
    otherwise an infinite product gives that infinity."""
    A = csr_rows([[(0, 1.0), (1, np.inf)], [(0, np.inf), (1, -np.inf)], [(0, 0.0), (1, np.inf)],
                  [(0, 1.0), (1, np.nan)], [(0, -2.0)], [(2, np.inf)]], 3)
    A = g.CSR(6, A.row_ptr, A.col_idx, A.val)
    x = np.array([1.0, 1.0, 0.0])
    y = pk.csr_spmv_exact(pk.CSR.from_host(A), to_dev(x)).cpu().numpy()
    assert y[0] == np.inf and np.isnan(y[1]) and y[2] == np.inf and np.isnan(y[3]) and y[4] == -2.0
    assert np.isnan(y[5])                                  # inf * 0
    assert same(y, spmv_exact(A, x))


@pytest.mark.parametrize("name", ["cd3d_128", "cd3d_256_var", "rand_1m"])
def test_exact_rows_full_size_sampled(name):
    p = g.problem(name)
    x = np.random.default_rng(4).uniform(-1, 1, p.A.n)
    y = pk.csr_spmv_exact(pk.CSR.from_host(p.A), to_dev(x)).cpu().numpy()
    rows = np.sort(np.random.default_rng(5).choice(p.A.n, size=20000, replace=False))
    assert same(y[rows], spmv_exact(p.A, x, rows=rows))
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,scale", [("cd2d_64", 24), ("cd3d_128", 10), ("rand_1m", 2000)])
@pytest.mark.parametrize("mode", [1, 2])
def test_solve_exact_rows_bitwise(name, scale, mode):
    """mode 1: r0, the true residual and replacement rows rounded once; mode 2: every A v
    as well.  Bit for bit against the oracle's solve with the same definitions."""
    p = g.problem(name, scale=scale)
    ex = solvers.default_dot(p.A.n)
    kw = {"resid": lambda A_, b_, x_: resid_exact(A_, b_, x_)}
    if mode == 2:
        kw["spmv"] = spmv_exact
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-10, max_iter=2000, dot=ex, **kw)
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-10, max_iter=2000, exact_rows=mode,
                       history=2000)
    assert info["status"] == ref.status == pk.OK
    assert info["iterations"] == ref.iterations
    assert np.array_equal(bits(info["history"]), bits(ref.history))
    assert np.array_equal(bits(x.cpu().numpy()), bits(ref.x))
    assert info["true_relres"] == ref.true_relres


def test_solve_exact_rows_hard_rows():
    """A few iterations from x0 on the mixed-path matrix: r0 = b - A x0 and every A v
    with exactly rounded rows, both row paths and the residual form on ties, wide
    exponents and subnormal products, bit for bit against the oracle."""
    A, x0, b = paths_case()
    ex = solvers.default_dot(A.n)
    ref = solvers.pbicgstab(A, b, x0=x0, tol=1e-300, max_iter=4, dot=ex, spmv=spmv_exact,
                            resid=lambda A_, b_, x_: resid_exact(A_, b_, x_))
    x, info = pk.solve(pk.CSR.from_host(A), to_dev(b), x0=to_dev(x0), tol=1e-300, max_iter=4, exact_rows=2,
                       history=4)
    assert info["status"] == ref.status
    assert info["iterations"] == ref.iterations
    assert np.array_equal(bits(info["history"]), bits(ref.history))
    assert np.array_equal(bits(x.cpu().numpy()), bits(ref.x))
    assert info["true_relres"] == ref.true_relres


def banded_paths_case():
    """A banded matrix (at most 7 offsets per 256-row slice, so the solver holds it in the
    offset form and the register path reads that form) with the value families of
    paths_case: narrow blocks, a block of wide exponents (LDS path), ties and cancellations,
    subnormal products, a ragged tail.  Returns (A, x0, b), all finite."""
    rng = np.random.default_rng(12)
    n = 1400
    offs = (-300, -17, -1, 0, 1, 17, 300)
    x = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-20, 20, n))
    x[900:1000] = rng.choice([1.0, -1.0, 0.5, 2.0 ** -53, 3.0], 100)
    x[1100:1200] = rng.uniform(-1, 1, 100) * 2.0 ** -540
    rows = []
    for i in range(n):
        cols = [i + d for d in offs if 0 <= i + d < n and (d == 0 or rng.random() > 0.02)]
        k = len(cols)
        blk = i // 256
        if blk == 1 or (blk == 4 and i % 3 == 0):
            vals = rng.standard_normal(k) * np.exp2(rng.integers(-90, 90, k))
        elif blk == 3:
            vals = rng.choice([1.0, -1.0, 2.0 ** 52, -(2.0 ** 52), 0.5], k)
        elif blk == 4 and i % 3 == 1:
            vals = rng.standard_normal(k) * 2.0 ** -540
        else:
            vals = rng.standard_normal(k)
        rows.append(list(zip(cols, vals.tolist())))
    A = csr_rows(rows, n)
    b = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-40, 40, n))
    b[768:1024] = rng.choice([0.0, 1.0, -2.0 ** -53, 2.0 ** 53], 256)
    return A, x, b


def test_solve_exact_rows_offset_form():
    """Exactly rounded rows read from the solver's offset form (the register path) and from
    CSR (the LDS path for rows spanning wide exponent ranges): a few iterations from x0 bit
    for bit against the oracle, and against the same solve on CSR (layout CSR)."""
    A, x0, b = banded_paths_case()
    ex = solvers.default_dot(A.n)
    ref = solvers.pbicgstab(A, b, x0=x0, tol=1e-300, max_iter=4, dot=ex, spmv=spmv_exact,
                            resid=lambda A_, b_, x_: resid_exact(A_, b_, x_))
    dA, db = pk.CSR.from_host(A), to_dev(b)
    x, info = pk.solve(dA, db, x0=to_dev(x0), tol=1e-300, max_iter=4, exact_rows=2, history=4)
    assert info["sliced"] & 64, info["sliced"]          # the offset form was built
    assert info["status"] == ref.status and info["iterations"] == ref.iterations
    assert np.array_equal(bits(info["history"]), bits(ref.history))
    assert np.array_equal(bits(x.cpu().numpy()), bits(ref.x))
    assert info["true_relres"] == ref.true_relres
    xc, ic = pk.solve(dA, db, x0=to_dev(x0), tol=1e-300, max_iter=4, exact_rows=2, layout=pk.LAYOUT_CSR)
    assert ic["sliced"] == 0
    assert np.array_equal(bits(xc.cpu().numpy()), bits(ref.x))


def test_exact_rows_replacement_and_history():
    p = g.problem("cd2d_64", scale=20)
    ex = solvers.default_dot(p.A.n)
    ref = solvers.pbicgstab(p.A, p.b, tol=1e-13, max_iter=150, dot=ex, spmv=spmv_exact, rr_period=10,
                            true_every=10, resid=lambda A_, b_, x_: resid_exact(A_, b_, x_))
    x, info = pk.solve(pk.CSR.from_host(p.A), to_dev(p.b), tol=1e-13, max_iter=150, exact_rows=2, rr_period=10,
                       true_every=10)
    assert info["iterations"] == ref.iterations
    assert np.array_equal(bits(info["true_history"]), bits(ref.true_history))
    assert np.array_equal(bits(x.cpu().numpy()), bits(ref.x))


def test_exact_rows_invalid_combinations():
    p = g.problem("cd2d_64", scale=8)
    A, b = pk.CSR.from_host(p.A), to_dev(p.b)
    for kw in ({"exact_rows": 3}, {"exact_rows": 1, "alg": pk.ALG_BICGSTAB},
               {"exact_rows": 2, "prec": pk.PREC_FP32_IR}, {"exact_rows": 1, "M": pk.jacobi(A)}):
        with pytest.raises(pk.LibError):
            pk.solve(A, b, **kw)
