"""Matrix Market loader (host side): the coordinate format in which the paper's test
matrices are distributed (Section 3, Table 1: SuiteSparse collection), read into the
CSR form the library takes (int32 row pointers and column indices, columns strictly
ascending within each row, FP64 values).

Supported headers: ``%%MatrixMarket matrix coordinate <field> <symmetry>`` with field
real, integer or pattern (pattern entries get the value 1) and symmetry general,
symmetric or skew-symmetric (the mirrored entry a_ji = a_ij, resp. -a_ij, is added for
every stored off-diagonal entry; a skew-symmetric file may not store diagonal entries).
Duplicate coordinates are summed (in file order, FP64).  Raises ValueError on: another
format (array, complex, hermitian), a matrix that is not square, an index outside
[1, n], a wrong entry count, or malformed lines.  No solver arithmetic happens here.
"""
from __future__ import annotations

import io
import os

import numpy as np


class Csr:
    """Host CSR (the same fields as synthgen.CSR)."""

    def __init__(self, n, row_ptr, col_idx, val):
        self.n, self.row_ptr, self.col_idx, self.val = int(n), row_ptr, col_idx, val

    @property
    def nnz(self) -> int:
        return int(self.col_idx.size)


def _open(src):
    if isinstance(src, (str, os.PathLike)):
        if str(src).endswith(".gz"):
            import gzip
            return io.TextIOWrapper(gzip.open(src, "rb"))
        return open(src, "r")
    return src


def read_matrix_market(src) -> Csr:
    """Read a square coordinate Matrix Market file (path, .gz path or text stream)."""
    fh = _open(src)
    try:
        header = fh.readline()
        parts = header.strip().split()
        if len(parts) != 5 or parts[0] != "%%MatrixMarket" or parts[1].lower() != "matrix":
            raise ValueError(f"not a Matrix Market matrix header: {header.strip()!r}")
        fmt, field, sym = (p.lower() for p in parts[2:])
        if fmt != "coordinate":
            raise ValueError(f"only the coordinate format is supported, not {fmt!r}")
        if field not in ("real", "integer", "pattern"):
            raise ValueError(f"unsupported field {field!r}")
        if sym not in ("general", "symmetric", "skew-symmetric"):
            raise ValueError(f"unsupported symmetry {sym!r}")
        line = fh.readline()
        while line and (line.startswith("%") or not line.strip()):
            line = fh.readline()
        size = line.split()
        if len(size) != 3:
            raise ValueError(f"bad size line: {line.strip()!r}")
        nr, nc, ne = (int(v) for v in size)
        if nr != nc:
            raise ValueError(f"matrix is not square: {nr} x {nc}")
        if nr < 0 or ne < 0:
            raise ValueError("negative size")
        if nr >= 2 ** 31:
            raise ValueError("n must be below 2^31")
        body = [l for l in fh.read().splitlines() if l.strip() and not l.lstrip().startswith("%")]
    finally:
        if fh is not src:
            fh.close()
    if len(body) != ne:
        raise ValueError(f"expected {ne} entries, found {len(body)}")
    ncol = 2 if field == "pattern" else 3
    rows = np.empty(ne, dtype=np.int64)
    cols = np.empty(ne, dtype=np.int64)
    vals = np.ones(ne, dtype=np.float64)
    for k, l in enumerate(body):
        f = l.split()
        if len(f) != ncol:
            raise ValueError(f"entry {k + 1}: expected {ncol} fields, got {l.strip()!r}")
        try:
            rows[k] = int(f[0])
            cols[k] = int(f[1])
            if field == "real":
                vals[k] = float(f[2])
            elif field == "integer":
                vals[k] = float(int(f[2]))
        except ValueError as e:
            raise ValueError(f"entry {k + 1}: {e}") from None
    if ne and (rows.min() < 1 or cols.min() < 1 or rows.max() > nr or cols.max() > nr):
        raise ValueError("index outside [1, n]")
    rows -= 1
    cols -= 1
    if sym != "general":
        off = rows != cols
        if sym == "skew-symmetric" and not np.all(off):
            raise ValueError("a skew-symmetric file stores no diagonal entries")
        mv = vals[off] if sym == "symmetric" else -vals[off]
        rows, cols, vals = (np.concatenate([rows, cols[off]]), np.concatenate([cols, rows[off]]),
                            np.concatenate([vals, mv]))
    return coo_to_csr(nr, rows, cols, vals)


def coo_to_csr(n, rows, cols, vals) -> Csr:
    """CSR from coordinates: entries ordered by (row, column), duplicates summed in their
    input order."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((np.arange(rows.size), cols, rows))   # stable: input order among duplicates
    r, c, v = rows[order], cols[order], vals[order]
    if r.size:
        first = np.concatenate([[True], (r[1:] != r[:-1]) | (c[1:] != c[:-1])])
        starts = np.nonzero(first)[0]
        ends = np.append(starts[1:], r.size)
        summed = v[starts].copy()
        for k in np.nonzero(ends - starts > 1)[0]:     # runs of duplicates: summed left to right
            acc = 0.0
            for t in v[starts[k]:ends[k]].tolist():
                acc += t
            summed[k] = acc
        r, c, v = r[starts], c[starts], summed
    if r.size >= 2 ** 31:
        raise ValueError("nnz must be below 2^31")
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    np.cumsum(rp, out=rp)
    return Csr(n, rp.astype(np.int32), c.astype(np.int32), v.astype(np.float64))


def write_matrix_market(path, A, comment: str = "") -> None:
    """Write a CSR as ``coordinate real general`` (values with 17 significant digits, so
    that they read back bit for bit)."""
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    with open(path, "w") as fh:
        fh.write("%%MatrixMarket matrix coordinate real general\n")
        for l in comment.splitlines():
            fh.write(f"% {l}\n")
        fh.write(f"{A.n} {A.n} {len(A.col_idx)}\n")
        for i, j, v in zip(rows.tolist(), np.asarray(A.col_idx).tolist(), np.asarray(A.val).tolist()):
            fh.write(f"{i + 1} {j + 1} {v!r}\n")
