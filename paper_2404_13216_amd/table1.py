"""Iteration counts of the paper's comparison (Section 3, Table 1) for matrices given as
Matrix Market files: BiCGStab, p-BiCGStab with ordinary FP64 dots, p-BiCGStab with exact
dots, and p-BiCGStab with residual replacement every k iterations, at two tolerances,
from x0 = 0 and without preconditioning, on the GPU.

The paper does not state its right-hand side; here b = A 1 (the all-ones solution).  The
stopping test is this library's: the true relative residual.  Usage:

    python -m paper_2404_13216_amd.table1 [--tols 1e-6,1e-9] [--rr 50] [--max-iter 10000] a.mtx [b.mtx ...]

prints one JSON line per matrix and a text table.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import ALG_BICGSTAB, CSR, DOTS_EXACT, DOTS_PLAIN, csr_spmv, csr_validate, solve
from .mtx import read_matrix_market

METHODS = [("BiCGStab", {"alg": ALG_BICGSTAB}), ("p-BiCGStab", {"dots": DOTS_PLAIN}),
           ("p-BiCGStab+exact", {"dots": DOTS_EXACT}), ("p-BiCGStabRR", {"dots": DOTS_PLAIN, "rr_period": None})]


def run_matrix(path, tols=(1e-6, 1e-9), rr=50, max_iter=10000, device="cuda"):
    import torch
    Ah = read_matrix_market(path)
    csr_validate(Ah)
    A = CSR.from_host(Ah, device)
    b = csr_spmv(A, torch.ones(Ah.n, dtype=torch.float64, device=device))   # b = A 1
    row = {"matrix": os.path.basename(path), "n": Ah.n, "nnz": Ah.nnz, "rhs": "A*1", "x0": "0", "runs": {}}
    for tol in tols:
        for name, kw in METHODS:
            kw = dict(kw)
            if "rr_period" in kw:
                kw["rr_period"] = rr
            x, info = solve(A, b, tol=tol, max_iter=max_iter, **kw)
            row["runs"][f"{name}@{tol:g}"] = {"iterations": info["iterations"], "status": info["status"],
                                              "true_relres": info["true_relres"]}
    return row


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("files", nargs="+")
    ap.add_argument("--tols", default="1e-6,1e-9")
    ap.add_argument("--rr", type=int, default=50, help="residual-replacement period k")
    ap.add_argument("--max-iter", type=int, default=10000)
    a = ap.parse_args(argv)
    tols = tuple(float(t) for t in a.tols.split(","))
    rows = [run_matrix(f, tols, a.rr, a.max_iter) for f in a.files]
    for r in rows:
        print(json.dumps(r))
    head = ["matrix"] + [f"{m}@{t:g}" for t in tols for m, _ in METHODS]
    print(" | ".join(head))
    for r in rows:
        cells = []
        for h in head[1:]:
            v = r["runs"][h]
            cells.append(str(v["iterations"]) if v["status"] == 0 else "-")
        print(" | ".join([r["matrix"]] + cells))
    return rows


if __name__ == "__main__":
    main()
