"""GPU sliced copies (csr_slice) vs the oracle.

The sliced layout stores slices of 256 rows column-major and pads each slice to its
longest row; one lane walks one row in storage order, so the products must be
bit-identical to the oracle's row-sequential SpMV (FP64, and FP32 with Dot2).  The
padded size is an integer fixed by the row lengths: it must equal the host count
exactly, and the copy is built exactly when that count is within nnz + nnz/8 + 256.
A solve with the sliced copy must return the same bits as one on CSR.
"""
import numpy as np
import pytest

import paper_2404_13216_amd as pk
import synthgen as g
from oracle import ctier
from oracle.spmv import spmv, spmv_f32
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def padded_entries(A):
    """Host count of the sliced size: 256 x the longest row of every slice of 256 rows."""
    lens = np.diff(A.row_ptr.astype(np.int64))
    ns = (A.n + 255) // 256
    lp = np.zeros(ns * 256, dtype=np.int64)
    lp[:A.n] = lens
    return int(256 * lp.reshape(ns, 256).max(axis=1).sum())


def expect_built(A):
    return padded_entries(A) <= A.nnz + A.nnz // 8 + 256


def max_spread(A):
    """Largest spread of col - row over the rows of one 256-row slice at one entry position
    (the solver's copy holds 16-bit residuals from each position's minimum when <= 65535)."""
    lens = np.diff(A.row_ptr.astype(np.int64))
    rows = np.repeat(np.arange(A.n, dtype=np.int64), lens)
    pos = np.arange(A.nnz, dtype=np.int64) - np.repeat(A.row_ptr[:-1].astype(np.int64), lens)
    d = A.col_idx.astype(np.int64) - rows
    key = (rows // 256) * (int(lens.max()) + 1 if A.nnz else 1) + pos
    if not A.nnz:
        return 0
    order = np.argsort(key, kind="stable")
    k, dv = key[order], d[order]
    starts = np.concatenate([[0], np.nonzero(np.diff(k))[0] + 1])
    return int((np.maximum.reduceat(dv, starts) - np.minimum.reduceat(dv, starts)).max())


def sorted_entries(A):
    """Host count of the row-sorted copy's size: rows ordered by decreasing length within
    windows of 4096, then 64 x the longest row of every group of 64 consecutive slots."""
    lens = np.diff(A.row_ptr.astype(np.int64))
    order = np.concatenate([np.sort(lens[a:a + 4096])[::-1] for a in range(0, A.n, 4096)] +
                           [np.zeros(0, dtype=np.int64)])
    nws = (A.n + 63) // 64
    lp = np.zeros(nws * 64, dtype=np.int64)
    lp[:A.n] = order
    return int(64 * lp.reshape(nws, 64).max(axis=1).sum()) if nws else 0


def ofs_slots(A):
    """Host count of the offset form's value slots: 256 x the number of distinct offsets
    col - row of every 256-row slice; None when some slice has more than 8 (or A has no
    entries)."""
    if A.nnz == 0:
        return None
    lens = np.diff(A.row_ptr.astype(np.int64))
    rows = np.repeat(np.arange(A.n, dtype=np.int64), lens)
    d = A.col_idx.astype(np.int64) - rows
    pairs = np.unique((rows // 256) * (1 << 33) + (d + (1 << 32)))
    cnt = np.bincount(pairs >> 33, minlength=(A.n + 255) // 256)
    return None if cnt.max() > 8 else int(256 * cnt.sum())


def expect_ofs(A):
    cap = A.nnz + A.nnz // 8 + 256
    t = ofs_slots(A)
    return t is not None and t <= cap and ((A.n + 255) // 256) * 256 <= 4 * cap


def expect_sliced_bits(A, layout=None):
    """info['sliced'] of a solve with layout AUTO, SLICED or SORTED: bit 0 when a copy of A
    is built, bit 2 when its column entries are 16-bit residuals, bit 4 when it is the
    row-sorted copy, bit 6 when it is the offset form (AUTO: when every slice has at most
    8 offsets, else as SLICED)."""
    cap = A.nnz + A.nnz // 8 + 256
    if layout in (None, pk.LAYOUT_AUTO) and expect_ofs(A):
        return 1 | 64
    if layout != pk.LAYOUT_SORTED:
        return (1 | (4 if max_spread(A) <= 65535 else 0)) if expect_built(A) else 0
    return (1 | 16) if sorted_entries(A) <= cap else 0


def with_long_range_entry(A, value):
    """A with one extra entry in row 0 at the last column (offset n - 1)."""
    k = int(A.row_ptr[1])
    ci = np.insert(A.col_idx, k, A.n - 1).astype(np.int32)
    val = np.insert(A.val, k, value)
    rp = A.row_ptr.astype(np.int64).copy()
    rp[1:] += 1
    return g.CSR(A.n, rp.astype(np.int32), ci, val)


def ragged(n, lens, seed):
    rng = np.random.default_rng(seed)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=int(k), replace=False)) for k in lens] +
                        [np.zeros(0, dtype=np.int64)]).astype(np.int32)
    return g.CSR(n, rp, ci, rng.standard_normal(int(rp[-1])))


def cases():
    out = [(name, g.problem(name, scale=sc).A) for name, sc in
           (("cd2d_64", None), ("cd3d_128", 20), ("cd3d_256_var", 17), ("spai_eval_128", 9), ("rand_1m", 50000))]
    rng = np.random.default_rng(7)
    # ragged tail (n not a multiple of 256), empty rows, lengths 6..7 (built)
    lens = rng.integers(6, 8, 1000)
    lens[::97] = 0
    out.append(("ragged_1000", ragged(1000, lens, 1)))
    out.append(("tiny_37", ragged(37, rng.integers(0, 2, 37), 2)))          # one partial slice (built)
    lens = rng.integers(5, 8, 1000)
    lens[::17] = 0
    out.append(("ragged_unbuilt", ragged(1000, lens, 5)))                     # padding above nnz/8 + 256
    out.append(("all_empty", ragged(300, np.zeros(300, dtype=np.int64), 3)))  # nnz = 0
    lens = np.full(2000, 4)
    lens[300] = 1500                                                          # one long row
    out.append(("one_long_row", ragged(2000, lens, 4)))
    return out


@pytest.mark.parametrize("name,A", cases(), ids=[c[0] for c in cases()])
def test_sliced_spmv_bitwise(name, A):
    dA = pk.CSR.from_host(A)
    S = pk.SlicedCSR(dA)
    assert S.entries == padded_entries(A)
    assert S.built == expect_built(A)
    x = np.random.default_rng(11).uniform(-1, 1, A.n)
    ref = spmv(A, x)
    if not S.built:
        with pytest.raises(pk.LibError):
            pk.csr_spmv_sliced(S, to_dev(x))
        return
    y = pk.csr_spmv_sliced(S, to_dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))
    y2 = pk.csr_spmv(dA, to_dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), y2.view(np.uint64))
    # FP32 values: the FP64-accumulating product and the Dot2 FP32 product
    import torch
    A32 = dA.with_values(dA.val.to(torch.float32))
    S32 = pk.SlicedCSR(A32)
    assert S32.built and S32.entries == S.entries
    A32h = g.CSR(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32).astype(np.float64))
    y = pk.csr_spmv_sliced(S32, to_dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), spmv(A32h, x).view(np.uint64))
    x32 = x.astype(np.float32)
    A32o = g.CSR(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32))
    y32 = pk.csr_spmv_f32_sliced(S32, to_dev(x32)).cpu().numpy()
    assert np.array_equal(y32.view(np.uint32), spmv_f32(A32o, x32).view(np.uint32))


def test_sliced_spmv_full_size_128():
    """128^3 (2,097,152 rows): every row bit-identical to the C oracle."""
    p = g.problem("cd3d_128")
    S = pk.SlicedCSR(pk.CSR.from_host(p.A))
    assert S.built and S.entries == padded_entries(p.A)
    x = np.random.default_rng(5).uniform(-1, 1, p.A.n)
    y = pk.csr_spmv_sliced(S, to_dev(x)).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), ctier.spmv(p.A, x).view(np.uint64))


@pytest.mark.parametrize("name,scale,prec", [("cd3d_128", 20, pk.PREC_FP64), ("cd2d_64", None, pk.PREC_FP64),
                                             ("cd3d_128", 20, pk.PREC_FP32_IR), ("rand_1m", 20000, pk.PREC_FP64)])
def test_solve_same_bits_with_and_without_slices(name, scale, prec):
    p = g.problem(name, scale=scale)
    A = pk.CSR.from_host(p.A)
    b = to_dev(p.b)
    xa, ia = pk.solve(A, b, tol=1e-10, prec=prec)
    xc, ic = pk.solve(A, b, tol=1e-10, prec=prec, layout=pk.LAYOUT_CSR)
    assert ia["sliced"] == expect_sliced_bits(p.A)
    assert ic["sliced"] == 0
    for k in ("status", "iterations", "outer_iterations", "true_checks"):
        assert ia[k] == ic[k], k
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))


def test_preconditioned_solve_slices_m():
    """Jacobi M (diagonal) and an M on A's pattern are sliced as well."""
    p = g.problem("cd3d_128", scale=20)
    A = pk.CSR.from_host(p.A)
    b = to_dev(p.b)
    J = pk.jacobi(A)
    xc, ic = pk.solve(A, b, M=J, tol=1e-10, layout=pk.LAYOUT_CSR)
    assert ic["sliced"] == 0
    # AUTO: both copies in the offset form; SLICED: both with 16-bit column residuals
    for layout, bits in ((pk.LAYOUT_AUTO, 1 | 2 | 64 | 128), (pk.LAYOUT_SLICED, 1 | 2 | 4 | 8)):
        xa, ia = pk.solve(A, b, M=J, tol=1e-10, layout=layout)
        assert ia["sliced"] == bits
        assert ia["iterations"] == ic["iterations"]
        assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))
    # M on A's pattern: scaled copy of A's values
    M = A.with_values(A.val * 0.5)
    xc, ic = pk.solve(A, b, M=M, tol=1e-10, max_iter=50, layout=pk.LAYOUT_CSR)
    for layout, bits in ((pk.LAYOUT_AUTO, 1 | 2 | 64 | 128), (pk.LAYOUT_SLICED, 1 | 2 | 4 | 8)):
        xa, ia = pk.solve(A, b, M=M, tol=1e-10, max_iter=50, layout=layout)
        assert ia["sliced"] == bits
        assert ia["status"] == ic["status"] and ia["iterations"] == ic["iterations"]
        assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("prec", [pk.PREC_FP64, pk.PREC_FP32_IR])
def test_solve_sliced_32bit_columns(prec):
    """One entry at offset n - 1 (spread above 65535 at its position) keeps the sliced
    copy's 32-bit columns; the solve must still return the same bits as on CSR (and as
    the oracle in FP64)."""
    p = g.problem("cd2d_64", scale=300)                    # n = 90,000
    Ah = with_long_range_entry(p.A, -1e-3 * p.A.val[0])
    assert max_spread(Ah) > 65535 and expect_built(Ah)
    assert max_spread(p.A) <= 65535 and expect_sliced_bits(p.A, pk.LAYOUT_SLICED) == 5
    xs = np.random.default_rng(3).uniform(-1, 1, Ah.n)
    bh = spmv(Ah, xs)
    A = pk.CSR.from_host(Ah)
    b = to_dev(bh)
    xa, ia = pk.solve(A, b, tol=1e-10, max_iter=60, prec=prec, layout=pk.LAYOUT_SLICED)
    xc, ic = pk.solve(A, b, tol=1e-10, max_iter=60, prec=prec, layout=pk.LAYOUT_CSR)
    assert ia["sliced"] == 1 and ic["sliced"] == 0
    assert ia["status"] == ic["status"] and ia["iterations"] == ic["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))
    if prec == pk.PREC_FP64:
        ora = ctier.pbicgstab(Ah, bh, tol=1e-10, max_iter=60)
        assert ora["iterations"] == ia["iterations"]
        assert np.array_equal(xa.cpu().numpy().view(np.uint64), ora["x"].view(np.uint64))


def dominant(A):
    """A with every row's diagonal entry set (inserted if absent) to 1 + sum |off-diagonal|."""
    rp, ci, va = [0], [], []
    for i in range(A.n):
        a, b = int(A.row_ptr[i]), int(A.row_ptr[i + 1])
        cols, vals = list(A.col_idx[a:b]), list(A.val[a:b])
        off = sum(abs(v) for c, v in zip(cols, vals) if c != i)
        if i in cols:
            vals[cols.index(i)] = 1.0 + off
        else:
            k = int(np.searchsorted(cols, i))
            cols.insert(k, i)
            vals.insert(k, 1.0 + off)
        ci += cols
        va += vals
        rp.append(len(ci))
    return g.CSR(A.n, np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32), np.array(va))


def wide_rows():
    """512 rows: the first slice 95..100 entries per row (more than 64 positions, so two
    groups of per-position bases), the second 3..5; a ragged tail of empty rows."""
    rng = np.random.default_rng(8)
    lens = np.concatenate([rng.integers(95, 101, 256), rng.integers(3, 6, 200), np.zeros(56, dtype=np.int64)])
    return ragged(512, lens, 6)


@pytest.mark.parametrize("name", ["ragged_1000", "wide_rows"])
def test_solve_ragged_16bit_residuals(name):
    """Ragged slices, a ragged tail, empty rows and rows longer than 64 entries through the
    solver's own sliced copy with 16-bit residuals: the same bits as on CSR and as the
    oracle."""
    A0 = wide_rows() if name == "wide_rows" else dict(cases())[name]
    Ah = dominant(A0)
    assert expect_sliced_bits(Ah) == 5, (name, max_spread(Ah), expect_built(Ah))   # too many offsets for AUTO's offset form
    xs = np.random.default_rng(9).uniform(-1, 1, Ah.n)
    bh = spmv(Ah, xs)
    A = pk.CSR.from_host(Ah)
    b = to_dev(bh)
    xa, ia = pk.solve(A, b, tol=1e-10, max_iter=8)
    xc, ic = pk.solve(A, b, tol=1e-10, max_iter=8, layout=pk.LAYOUT_CSR)
    assert ia["sliced"] == 5 and ic["sliced"] == 0
    assert ia["status"] == ic["status"] and ia["iterations"] == ic["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))
    ora = ctier.pbicgstab(Ah, bh, tol=1e-10, max_iter=8)
    assert ora["iterations"] == ia["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), ora["x"].view(np.uint64))


def sorted_cases():
    rng = np.random.default_rng(12)
    out = [(n, a) for n, a in cases() if n in ("ragged_1000", "tiny_37", "ragged_unbuilt", "one_long_row")]
    lens = rng.integers(0, 300, 2 * 4096 + 37)              # two sort windows and a ragged third
    lens[::13] = 0
    out.append(("windows_8229", ragged(2 * 4096 + 37, lens, 13)))
    out.append(("rand_50000", g.problem("rand_1m", scale=50000).A))
    out.append(("cd2d_64", g.problem("cd2d_64").A))
    return out


@pytest.mark.parametrize("name,A0", sorted_cases(), ids=[c[0] for c in sorted_cases()])
def test_solve_row_sorted_bitwise(name, A0):
    """The row-sorted copy (64-row slices of rows ordered by length within windows of 4096
    rows, a permutation back to the row order): ragged windows, empty rows, one very long
    row; the same bits as on CSR and as the oracle, FP64 and FP32 refinement."""
    Ah = dominant(A0)
    want = expect_sliced_bits(Ah, pk.LAYOUT_SORTED)
    # one row of 1500 entries pads its 64-row slice past nnz + nnz/8 + 256: CSR is kept
    assert want == (0 if name == "one_long_row" else 17), (name, sorted_entries(Ah), Ah.nnz)
    xs = np.random.default_rng(9).uniform(-1, 1, Ah.n)
    bh = spmv(Ah, xs)
    A = pk.CSR.from_host(Ah)
    b = to_dev(bh)
    xa, ia = pk.solve(A, b, tol=1e-10, max_iter=8, layout=pk.LAYOUT_SORTED)
    xc, ic = pk.solve(A, b, tol=1e-10, max_iter=8, layout=pk.LAYOUT_CSR)
    assert ia["sliced"] == want and ic["sliced"] == 0
    assert ia["status"] == ic["status"] and ia["iterations"] == ic["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))
    ora = ctier.pbicgstab(Ah, bh, tol=1e-10, max_iter=8)
    assert ora["iterations"] == ia["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), ora["x"].view(np.uint64))
    # to convergence, and the FP32 refinement (Dot2 FP32 SpMV on the sorted copy)
    for prec in (pk.PREC_FP64, pk.PREC_FP32_IR):
        xa, ia = pk.solve(A, b, tol=1e-10, prec=prec, layout=pk.LAYOUT_SORTED)
        xc, ic = pk.solve(A, b, tol=1e-10, prec=prec, layout=pk.LAYOUT_CSR)
        for k in ("status", "iterations", "outer_iterations", "true_checks"):
            assert ia[k] == ic[k], (prec, k)
        assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64)), prec


def test_row_sorted_preconditioner():
    """SORTED on the random family (the 256-row copy would need 4.5x padding), for A and
    for an M on A's pattern; same bits as on CSR (which AUTO keeps there)."""
    p = g.problem("rand_1m", scale=30000)
    assert not expect_built(p.A) and expect_sliced_bits(p.A) == 0
    assert expect_sliced_bits(p.A, pk.LAYOUT_SORTED) == 17
    A = pk.CSR.from_host(p.A)
    b = to_dev(p.b)
    d = 1.0 / p.A.diag()
    rows = np.repeat(np.arange(p.A.n), np.diff(p.A.row_ptr))
    mv = np.where(rows == p.A.col_idx, d[rows], 1e-3 * d[rows])
    M = A.with_values(to_dev(mv))
    xa, ia = pk.solve(A, b, M=M, tol=1e-10, max_iter=40, layout=pk.LAYOUT_SORTED)
    xc, ic = pk.solve(A, b, M=M, tol=1e-10, max_iter=40, layout=pk.LAYOUT_CSR)
    assert ia["sliced"] == 1 | 2 | 16 | 32 and ic["sliced"] == 0
    assert ia["status"] == ic["status"] and ia["iterations"] == ic["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))


def banded(n, offsets, seed, drop=0.03, extra=None):
    """Rows with entries at row + d for d in `offsets` (inside [0, n)), each dropped with
    probability `drop` (the diagonal kept), every 41st row empty but its diagonal; `extra`:
    (row, offset) entries added to make one slice exceed 8 offsets."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        cols = [i + d for d in offsets if 0 <= i + d < n and (d == 0 or (i % 41 and rng.random() >= drop))]
        if extra and i == extra[0]:
            cols.append(i + extra[1])
        cols = sorted(set(cols))
        rows.append([(c, float(rng.standard_normal())) for c in cols])
    rp, ci, va = [0], [], []
    for r in rows:
        ci += [c for c, _ in r]
        va += [v for _, v in r]
        rp.append(len(ci))
    return dominant(g.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va)))


def offset_cases():
    offs8 = (-300, -17, -1, 0, 1, 17, 300, 512)
    return [("cd2d_64", g.problem("cd2d_64").A), ("cd3d_128_s20", g.problem("cd3d_128", scale=20).A),
            ("cd3d_256_var_s17", g.problem("cd3d_256_var", scale=17).A),
            ("spai_eval_128_s9", g.problem("spai_eval_128", scale=9).A),
            ("banded8_1000", banded(1000, offs8, 21)),                            # 8 offsets, ragged tail
            ("banded5_700", banded(700, (-40, -1, 0, 1, 40), 22)),
            ("banded9_1000", banded(1000, offs8, 23, extra=(300, 650))),           # slice 1: 9 offsets
            ("banded8_sparse", banded(1000, offs8, 24, drop=0.3))]                 # slots above nnz/8 + 256


@pytest.mark.parametrize("name,Ah", offset_cases(), ids=[c[0] for c in offset_cases()])
def test_solve_offset_form_bitwise(name, Ah):
    """The offset form (per slice the offsets col - row, per row a mask byte and one value
    slot per offset): stencils with their boundary rows, banded rows with random missing
    entries and empty rows, a ragged tail; a slice with 9 offsets, and slots beyond
    nnz + nnz/8 + 256, keep the column form.
    Same bits as on CSR and as the oracle: 8 iterations, then to convergence in FP64, the
    FP32 refinement (Dot2 FP32 SpMV on the form) and the FP32-matrix form."""
    want = expect_sliced_bits(Ah)
    assert (want == 65) == (name not in ("banded9_1000", "banded8_sparse")), (name, ofs_slots(Ah))
    xs = np.random.default_rng(9).uniform(-1, 1, Ah.n)
    bh = spmv(Ah, xs)
    A = pk.CSR.from_host(Ah)
    b = to_dev(bh)
    xa, ia = pk.solve(A, b, tol=1e-10, max_iter=8)
    xc, ic = pk.solve(A, b, tol=1e-10, max_iter=8, layout=pk.LAYOUT_CSR)
    assert ia["sliced"] == want and ic["sliced"] == 0
    if want == 65:
        assert ia["sliced_entries"] == ofs_slots(Ah)
    assert ia["status"] == ic["status"] and ia["iterations"] == ic["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64))
    ora = ctier.pbicgstab(Ah, bh, tol=1e-10, max_iter=8)
    assert ora["iterations"] == ia["iterations"]
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), ora["x"].view(np.uint64))
    for prec in (pk.PREC_FP64, pk.PREC_FP32_IR, pk.PREC_FP32_MATRIX):
        xa, ia = pk.solve(A, b, tol=1e-10, prec=prec, max_iter=3000)
        xc, ic = pk.solve(A, b, tol=1e-10, prec=prec, max_iter=3000, layout=pk.LAYOUT_CSR)
        assert ia["sliced"] & 65 == want & 65
        for k in ("status", "iterations", "outer_iterations", "true_checks"):
            assert ia[k] == ic[k], (prec, k)
        assert np.array_equal(xa.cpu().numpy().view(np.uint64), xc.cpu().numpy().view(np.uint64)), prec
