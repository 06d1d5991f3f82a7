#!/usr/bin/env python3
"""Benchmark: time to true relative residual 1e-10, plus SpMV / exact-dot HBM bandwidth.

Headline workload (the largest single-GPU configuration): 3D upwind convection-diffusion
on a 256^3 grid, 7-point stencil, cell-wise diffusivity exp(N(0,1)) (harmonic face
means), velocity (50, 25, 10), n = 16,777,216, nnz = 117,047,296, CSR FP64 with int32
indices; x* ~ U[-1, 1] (seed 3), b = A x*, x0 = 0, tol 1e-10 on the true relative
residual.  One step = one complete FP64 p-BiCGStab solve with exact dot products
(initialisation, every iteration's phase A / SpMV / phase B / SpMV with their fused exact
dots, and the true-residual checks), inputs already resident in HBM.  Its matrix (1.17 GB
in the solver's sliced copy) and Krylov vectors (1.6 GB) are far larger than the 256 MB
Infinity Cache, so every iteration streams from HBM: the roofline is HBM bandwidth.

Also reported (outside the timed steps):
  * on the headline matrix: BiCGStab, p-BiCGStab with residual replacement every 50
    iterations, FP32 refinement with reliable updates at update threshold 0.1 (the
    library default) and 1e-5, each against the fastest FP64 form that reaches 1e-10;
  * per-kernel durations of the solve's four kernels (phase A, v = A z, phase B, t = A w)
    from HIP events that the kernels' own dispatches stamp inside a solve identical to
    the timed ones, and from them the roofline of the dominant kernel (the SpMV);
  * the 128^3 constant-coefficient workload, whose 146 MB sliced matrix stays resident in
    the Infinity Cache (its SpMV figures are cache bandwidth, not HBM), with its own
    kernel table, forms, and the paper's central comparison (exact vs ordinary FP64
    dots, with and without residual replacement, at 1e-10 and 1e-13);
  * the 64^2 workload (n = 4096): wall time only (latency-bound);
  * the random unsymmetric n = 10^6 matrix: FP64 forms vs FP32 refinement;
  * the learned preconditioner: training on the seeded matrices 100..299 with the GPU
    kernels, then the held-out 128^3 Peclet-50 matrix solved plain, with Jacobi and with
    the learned M (setup time stated separately);
  * micro-benchmarks (HIP events around every launch): the SpMV kernel shapes on a cold
    cache and the standalone exact dot;
  * the CPU oracle (C, exact dots) on the headline workload on this host's cores, all
    threads and one thread: a bounded sample of iterations, extrapolated per iteration to
    the GPU's iteration count.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--solve-only]
                       [--legs cd3d_128,claim,cd2d_64,learned,rand_1m] [--epochs 30]
                       [--traffic-run [--workload cd3d_256_var|cd3d_128]] [--infer-run]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_2404_13216_amd", "csrc")
HEADLINE = "cd3d_256_var"
WORKLOAD_DESC = {"cd3d_256_var": "cd3d_256_var: 3D upwind convection-diffusion 256^3, kappa=exp(N(0,1)) cell-wise "
                                  "(harmonic faces), v=(50,25,10), seed 3",
                 "cd3d_128": "cd3d_128: 3D upwind convection-diffusion 128^3, v=(30,20,10), seed 1 "
                             "(Infinity-Cache-resident matrix)"}
TRAFFIC_FILES = {"cd3d_256_var": os.path.join(ROOT, "profiles", "hbm_traffic_cd3d_256_var.md"),
                 "cd3d_128": os.path.join(ROOT, "profiles", "hbm_traffic_cd3d_128.md")}
KEV = 128  # iterations of each timed solve whose kernels carry timing events


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of what determines the HBM traffic the counter profile records: the kernel
    sources and the launch-shape constants of the host launchers (the driver logic in
    capi.hip and the learned-preconditioner kernels in spai.hip do not change it)."""
    h = hashlib.sha256()
    for f in ("kernels.hpp", "state.hpp", "xdot.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(CSRC, "capi.hip")) as fh:
        for line in fh:
            if line.startswith("constexpr int") and ("GRID" in line or "BLOCK" in line or "WORKERS" in line
                                                    or "KEXP" in line):
                h.update(line.encode())
    return h.hexdigest()[:16]


_SLEEP_CYCLES_PER_S = None


def hold_stream(torch, seconds):
    """Enqueue a device-side spin of about `seconds` on the current stream, so that the
    launches the host enqueues behind it start back to back: event timings then measure
    device time, not the host's launch latency (a ctypes call costs tens of microseconds,
    longer than some of the kernels it launches)."""
    global _SLEEP_CYCLES_PER_S
    if _SLEEP_CYCLES_PER_S is None:
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(1000)
        s.record()
        torch.cuda._sleep(1 << 20)
        e.record()
        e.synchronize()
        _SLEEP_CYCLES_PER_S = (1 << 20) / max(s.elapsed_time(e) / 1e3, 1e-6)
    torch.cuda._sleep(int(seconds * _SLEEP_CYCLES_PER_S))


def time_launches(fn, reps, torch):
    """Median duration of fn() over `reps` back-to-back launches, each bracketed by HIP
    events on the current stream, all queued behind a device-side hold."""
    fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    hold_stream(torch, 2e-3 + reps * 1e-4)
    ev[0].record()
    for k in range(reps):
        fn()
        ev[k + 1].record()
    ev[-1].synchronize()
    return float(np.median([ev[k].elapsed_time(ev[k + 1]) / 1e3 for k in range(reps)]))


def spmv_cold(pk, torch, A, reps, kind=None, S=None):
    """Median duration of one SpMV launch with a 1 GiB read before each (no launch is
    served from the Infinity Cache, and no dirty lines are left to write back); returns
    (seconds, GB/s of 12 B/nnz + 20 B/row).  With S (a built sliced copy of A) the sliced
    row-sequential kernel is timed."""
    flush = torch.ones(128 << 20, dtype=torch.float64, device=A.val.device)
    vin = torch.ones(A.n, dtype=torch.float64, device=A.val.device)
    vout = torch.empty_like(vin)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for it in range(reps + 1):
        flush.sum()
        e0.record()
        if S is not None:
            pk.csr_spmv_sliced(S, vin, vout)
        else:
            pk.csr_spmv(A, vin, vout, kind=kind)
        e1.record()
        e1.synchronize()
        if it:
            ts.append(e0.elapsed_time(e1) / 1e3)
    dt = float(np.median(ts))
    vb = 12 if A.val.dtype == torch.float64 else 8
    return dt, ((vb * A.nnz + 20 * A.n) / dt / 1e9)


def timed_solve(pk, torch, A, b, reps=1, **opts):
    """One untimed solve, then `reps` solves from x0 = 0, each bracketed by device
    synchronisations; returns (median seconds, info of the last solve, x)."""
    solver = pk.Solver(A, **opts)
    x = torch.zeros(A.n, dtype=torch.float64, device=b.device)
    solver.solve(b, x)
    secs = []
    for _ in range(reps):
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = solver.solve(b, x)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t)
    return float(np.median(secs)), info, x


def rel(torch, a, b):
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def fp64_forms(pk, torch, A, b, xs, reps, plain=None):
    """The FP64 solves of one workload: plain p-BiCGStab (exact dots; given, or timed
    here), p-BiCGStab with residual replacement every 50 iterations, and BiCGStab
    (Algorithm 1).  Returns (forms, x of the plain solve)."""
    forms = {}
    if plain is None:
        plain = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000)
    t64, i64, x64 = plain
    forms["pbicgstab_fp64"] = {"seconds": t64, "iterations": i64["iterations"], "true_relres": i64["true_relres"],
                               "status": i64["status"], "rel_err_vs_xstar": rel(torch, x64, xs)}
    for key, kw in (("pbicgstab_fp64_rr50", {"rr_period": 50}), ("bicgstab_fp64", {"alg": pk.ALG_BICGSTAB})):
        tr, ir, xr = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000, **kw)
        forms[key] = {"seconds": tr, "iterations": ir["iterations"], "true_relres": ir["true_relres"],
                      "status": ir["status"], "rel_err_vs_xstar": rel(torch, xr, xs)}
        log(f"  {key}: {tr:.4f} s, {ir['iterations']} iterations, status {ir['status']}")
    return forms, x64


def converged(f):
    return f["status"] == 0 and f["true_relres"] <= 1e-10


def precision_forms(pk, torch, A, b, xs, x64, forms, reps):
    """FP32 refinement with reliable updates at the default update threshold (0.1) and at
    1e-5, and the FP32-matrix form (FP32 values, FP64 vectors, replacement against the
    FP64 A every 50 iterations), each with its error against the plain FP64 solution and
    x*, beside the FP64 forms.  speedup_vs_fp64 compares with plain FP64 p-BiCGStab and is null when that
    solve did not reach 1e-10; speedup_vs_fastest_fp64 compares with the fastest FP64
    form that did."""
    ok = {k: v for k, v in forms.items() if converged(v)}
    fastest = min(ok, key=lambda k: ok[k]["seconds"]) if ok else None
    t64 = forms["pbicgstab_fp64"]["seconds"] if converged(forms["pbicgstab_fp64"]) else None
    out = {}
    for key, itol in (("fp32_ir", None), ("fp32_ir_inner_1e-5", 1e-5), ("fp32_matrix", None)):
        kw = {} if itol is None else {"inner_tol": itol}
        prec = pk.PREC_FP32_MATRIX if key == "fp32_matrix" else pk.PREC_FP32_IR
        ti, ii, xi = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000, prec=prec, **kw)
        out[key] = {"seconds": ti, "inner_tol": (itol or 0.1) if prec == pk.PREC_FP32_IR else None,
                    "inner_iterations": ii["iterations"],
                    "outer": ii["outer_iterations"], "fell_back_to_fp64": ii["fell_back"],
                    "true_relres": ii["true_relres"], "status": ii["status"],
                    "rel_diff_vs_fp64_solve": rel(torch, xi, x64), "rel_err_vs_xstar": rel(torch, xi, xs),
                    "speedup_vs_fp64": (t64 / ti) if t64 else None,
                    "fastest_fp64": fastest,
                    "speedup_vs_fastest_fp64": (ok[fastest]["seconds"] / ti) if fastest else None}
        log(f"  {key}: {ti:.4f} s, {ii['iterations']} FP32 iterations, fell back {ii['fell_back']}, "
            f"status {ii['status']}")
    return out


def kernel_table(pk, torch, A, b, n, nnz, info, x, batch):
    """Durations of the solve's four kernels over iterations 1..KEV of one more solve,
    identical to the timed ones, whose kernels carry HIP events stamped by their own
    dispatches (hipExtLaunchKernel: no markers between kernels, the launches keep their
    spacing).  Bytes per launch: the algorithmic figures -- 12 per nonzero + 20 per row
    for an SpMV (8-byte value, 4-byte column index; x once, y, row pointers), 104 and 80
    per row for the phases -- and, for the SpMV, what the solve's layout moves
    (layout_bytes)."""
    tsolver = pk.Solver(A, kernel_events=KEV, tol=1e-10, max_iter=10000)
    xk = torch.zeros(n, dtype=torch.float64, device=b.device)
    _, kinfo = tsolver.solve(b, xk)
    assert kinfo["iterations"] == info["iterations"] and torch.equal(xk, x)
    ktimes = tsolver.kernel_times()
    del tsolver, xk
    used = max(1, min(KEV, info["iterations"] - 2 * batch))
    spmv_alg = 12 * nnz + 20 * n
    spmv_layout = layout_bytes(info, nnz, n)
    roles = {"phase_a": 104 * n, "spmv_az": spmv_alg, "phase_b": 80 * n, "spmv_aw": spmv_alg}
    kern = {}
    for name, nb in roles.items():
        ts = np.array(ktimes[name][:used])
        kern[name] = {"us": float(ts.mean() * 1e6), "median_us": float(np.median(ts) * 1e6),
                      "min_us": float(ts.min() * 1e6), "max_us": float(ts.max() * 1e6),
                      "bytes": nb, "GBs": nb / ts.mean() / 1e9, "launches": int(ts.size)}
    both = np.array(ktimes["spmv_az"][:used] + ktimes["spmv_aw"][:used])
    kern["spmv_seq"] = {"us": float(both.mean() * 1e6), "median_us": float(np.median(both) * 1e6),
                        "bytes": spmv_alg, "GBs": spmv_alg / both.mean() / 1e9, "launches": int(both.size),
                        "layout": layout_name(info),
                        "layout_bytes": spmv_layout, "layout_GBs": spmv_layout / both.mean() / 1e9}
    for v in kern.values():
        v["frac_of_peak"] = v["GBs"] / HBM_PEAK_GBS
    return kern, used, sum(kern[k]["us"] for k in roles)


def layout_name(info):
    sl = info["sliced"]
    if not sl & 1:
        return "csr"
    if sl & 64:
        return "offset form (256-row slices, per-row slot mask)"
    if sl & 16:
        return "row-sorted sliced copy"
    return "sliced copy (256-row slices%s)" % (", 16-bit column residuals" if sl & 4 else "")


def layout_bytes(info, nnz, n):
    """Bytes one SpMV of the solve moves with its layout: values (8 per stored slot), column
    entries (4, or 2 as 16-bit residuals; none in the offset form, which reads a mask byte
    per row and no row pointers), x once and y (8 + 8 per row), row pointers (4 per row)."""
    sl, ent = info["sliced"], info.get("sliced_entries", 0)
    if not sl & 1:
        return 12 * nnz + 20 * n
    if sl & 64:
        return 8 * ent + 17 * n
    col_bytes = 2 if sl & 4 else 4
    return (8 + col_bytes) * ent + 20 * n


def config_leg(pk, torch, g, dev, name, reps):
    """FP64 forms vs FP32 refinement on another workload (time to true relative residual
    1e-10), plus its SpMV kernel shapes on a cold cache."""
    t0 = time.time()
    prob = g.problem(name)
    A = pk.CSR.from_host(prob.A, dev)
    b = torch.from_numpy(prob.b).to(dev)
    xs = torch.from_numpy(prob.xstar).to(dev)
    gen = time.time() - t0
    forms, x64 = fp64_forms(pk, torch, A, b, xs, reps)
    forms.update(precision_forms(pk, torch, A, b, xs, x64, forms, reps))
    out = {"n": prob.A.n, "nnz": prob.A.nnz, "host_generation_s": gen, "forms": forms}
    kern = {}
    S = pk.SlicedCSR(A)
    out["sliced"] = {"built": S.built, "entries": S.entries}
    shapes = [("spmv_seq_cold", pk.SPMV_SEQ, None), ("spmv_vector_cold", pk.SPMV_VECTOR, None)]
    if S.built:
        shapes.insert(0, ("spmv_seq_sliced_cold", pk.SPMV_SEQ, S))
    for kname, kind, sl in shapes:
        dt, gbs = spmv_cold(pk, torch, A, 20, kind, sl)
        kern[kname] = {"us": dt * 1e6, "GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    out["kernels"] = kern
    del S
    log(f"{name}:", json.dumps(out))
    return out


def small_leg(pk, torch, g, dev, reps=20):
    """The 64^2 workload (n = 4096, 20,224 nonzeros): latency-bound, wall time only."""
    prob = g.problem("cd2d_64")
    A = pk.CSR.from_host(prob.A, dev)
    b = torch.from_numpy(prob.b).to(dev)
    out = {}
    for key, kw in (("pbicgstab_fp64", {}), ("bicgstab_fp64", {"alg": pk.ALG_BICGSTAB}),
                    ("fp32_ir", {"prec": pk.PREC_FP32_IR})):
        t, info, _ = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=2000, **kw)
        out[key] = {"seconds": t, "iterations": info["iterations"], "status": info["status"],
                    "true_relres": info["true_relres"], "us_per_iteration": t / max(info["iterations"], 1) * 1e6}
    log("cd2d_64:", json.dumps(out))
    return out


def claim_leg(pk, torch, A, b, n):
    """The paper's central comparison on the benchmark matrix: exact vs ordinary FP64
    dots, without and with residual replacement (period 50), at the benchmark tolerance
    1e-10 and at 1e-13 (below what the recurrences sustain); iteration cap 1500.  For
    the 1e-13 runs the true residual is recorded every 10 iterations (bit-identical to
    the oracle's) and its minimum is reported: the attainable accuracy.  "exact_rows" runs
    round every SpMV row and every residual row once as well (no summation order left
    anywhere in the solve): whether the floor comes from the SpMV's rounding."""
    out = {}
    for tol in (1e-10, 1e-13):
        for label, dots, rr, xr in (("exact", pk.DOTS_EXACT, 0, 0), ("plain", pk.DOTS_PLAIN, 0, 0),
                                    ("exact_rr50", pk.DOTS_EXACT, 50, 0), ("plain_rr50", pk.DOTS_PLAIN, 50, 0),
                                    ("exact_rows", pk.DOTS_EXACT, 0, 2)):
            every = 10 if tol < 1e-12 else 0
            solver = pk.Solver(A, tol=tol, max_iter=1500, dots=dots, rr_period=rr, true_every=every,
                               exact_rows=xr)
            x = torch.zeros(n, dtype=torch.float64, device=b.device)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = solver.solve(b, x)
            torch.cuda.synchronize()
            t = time.perf_counter() - t
            row = {"seconds": t, "status": info["status"], "iterations": info["iterations"],
                   "true_checks": info["true_checks"], "true_relres": info["true_relres"],
                   "rec_relres": info["rec_relres"]}
            if every:
                th = solver.true_history.cpu().numpy()
                th = th[~np.isnan(th)]
                if th.size:
                    k = int(np.argmin(th))
                    row["min_true_relres"] = float(th[k])
                    row["min_true_at_iteration"] = (k + 1) * every
            out[f"{label}_tol{tol:g}"] = row
    log("claim:", json.dumps(out))
    return out


def learned_leg(pk, torch, g, dev, reps, epochs):
    """Learned SPAI: train on the seeded matrices 100..299 (2D/3D convection-diffusion,
    n 16k-262k, Peclet 1-100, kappa = exp(N(0,1))) with the GPU forward / backward / Adam
    kernels, then solve the held-out 128^3 Peclet-50 matrix (seed 4) unpreconditioned,
    with Jacobi, and with the learned M (bf16 inference, FP32 values, fallback on)."""
    from paper_2404_13216_amd import spai
    t0 = time.time()
    train = [g.training_problem(s) for s in range(100, 300)]
    gen = time.time() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params, hist = spai.train(train, epochs=epochs, lr=1e-3, seed=0, device=dev)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    train_rows = sum(p.A.n for p in train)
    train_nnz = sum(p.A.nnz for p in train)
    del train
    torch.cuda.empty_cache()
    ev = g.problem("spai_eval_128")
    A = pk.CSR.from_host(ev.A, dev)
    b = torch.from_numpy(ev.b).to(dev)
    xs = torch.from_numpy(ev.xstar).to(dev)
    t_plain, ip, xp = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000)
    t0 = time.perf_counter()
    J = pk.jacobi(A, torch.float32)
    torch.cuda.synchronize()
    t_jset = time.perf_counter() - t0
    t_jac, ij, xj = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000, M=J, fallback=1)
    # setup: features (one pass over A) and bf16 inference of the 5,057-parameter MLP per nonzero
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sm = spai.SpaiMatrix(A)
    M = sm.preconditioner(params)
    torch.cuda.synchronize()
    t_set = time.perf_counter() - t0
    t_inf = time_launches(lambda: sm.m_bf16(params), 10, torch)
    t_ln, il, xl = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000, M=M, fallback=1)

    def row(t, info, x, setup=0.0):
        return {"seconds": t, "seconds_incl_setup": t + setup, "iterations": info["iterations"],
                "true_relres": info["true_relres"], "status": info["status"], "fell_back": info["fell_back"],
                "rel_err_vs_xstar": rel(torch, x, xs), "rel_diff_vs_plain": rel(torch, x, xp)}
    out = {"workload": "spai_eval_128: 3D convection-diffusion 128^3, Peclet 50 (direction from seed 4), "
                       "kappa = exp(N(0,1)); n=%d nnz=%d" % (ev.A.n, ev.A.nnz),
           "training": {"matrices": 200, "seeds": "100-299", "rows": train_rows, "nnz": train_nnz,
                        "epochs": epochs, "steps": epochs * 200, "optimizer": "Adam lr 1e-3",
                        "host_generation_s": gen, "gpu_training_s": t_train,
                        "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]},
           "plain": row(t_plain, ip, xp),
           "jacobi": row(t_jac, ij, xj, t_jset),
           "learned": row(t_ln, il, xl, t_set),
           "learned_setup_s": t_set,
           "bf16_inference_us": t_inf * 1e6,
           "bf16_inference_tflops": ev.A.nnz * 2 * (12 * 64 + 64 * 64 + 64) / t_inf / 1e12}
    out["learned"]["speedup_vs_plain"] = t_plain / t_ln
    out["learned"]["speedup_vs_plain_incl_setup"] = t_plain / (t_ln + t_set)
    out["jacobi"]["speedup_vs_plain"] = t_plain / t_jac
    log("learned:", json.dumps(out))
    return out


def traffic_run(pk, torch, A, b, n, nnz, dev):
    """Kernels whose HBM bytes rocprofv3 counters measure: a 256 MiB device copy (the
    calibration: 256 MiB read, 256 MiB written), the SpMV, phase A / phase B and the
    standalone exact dot on the chosen workload, each launched 10 times with a 1 GiB read
    between launches so that no launch is served from the Infinity Cache; then one
    complete solve, whose kernels run as in the timed steps."""
    log(f"source_hash {kernel_source_hash()}")
    rng = np.random.default_rng(1)
    V = {k: torch.from_numpy(rng.standard_normal(n) * 1e-3).to(dev) for k in
         ("x", "r", "rhat", "w", "t", "p", "s", "z", "q", "y", "v")}
    scal = torch.tensor([0.5, 0.25, 0.75], dtype=torch.float64, device=dev)
    dots = torch.empty(4, dtype=torch.float64, device=dev)
    wsp = torch.empty(pk.lib().pbcg_phase_workspace_bytes(n), dtype=torch.uint8, device=dev)
    src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    flush = torch.ones(128 << 20, dtype=torch.float64, device=dev)
    o1 = torch.empty(1, dtype=torch.float64, device=dev)
    wse = torch.empty(pk.lib().exdot_workspace_bytes(n), dtype=torch.uint8, device=dev)
    S = pk.SlicedCSR(A)   # the solve's SpMV reads the sliced copy when one is built
    for _ in range(10):
        flush.sum()
        dst.copy_(src)
        flush.sum()
        if S.built:
            pk.csr_spmv_sliced(S, V["z"], V["v"])
        else:
            pk.csr_spmv(A, V["z"], V["v"])
        flush.sum()
        pk.pbcg_phase_a(V, scal, False, dots, wsp)
        flush.sum()
        pk.pbcg_phase_b(V, scal, dots, wsp)
        flush.sum()
        pk.exdot(V["r"], V["w"], o1, wse)
    torch.cuda.synchronize()
    del V, S, flush, src, dst
    torch.cuda.empty_cache()
    solver = pk.Solver(A, tol=1e-10, max_iter=10000)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    _, info = solver.solve(b, x)
    torch.cuda.synchronize()
    log(f"traffic run done (solve: {info['iterations']} iterations, status {info['status']}, "
        f"layout {layout_name(info)}, layout_bytes {layout_bytes(info, nnz, n)})")


def infer_run(pk, torch, g, dev):
    """The bf16 inference kernel alone, for rocprofv3 counter runs: the held-out 128^3
    matrix's features, the 5,057 MLP parameters drawn from a seeded N(0, 0.05^2) (the
    kernel's work does not depend on their values: no data-dependent branches), 10
    launches."""
    from paper_2404_13216_amd import spai
    ev = g.problem("spai_eval_128")
    A = pk.CSR.from_host(ev.A, dev)
    sm = spai.SpaiMatrix(A)
    nparam = pk.lib().spai_param_count()
    params = torch.from_numpy((np.random.default_rng(0).standard_normal(nparam) * 0.05).astype(np.float32)).to(dev)
    for _ in range(10):
        sm.m_bf16(params)
    torch.cuda.synchronize()
    log(f"infer run done (nnz {ev.A.nnz}, 10 launches)")


def resident_leg(pk, torch, g, dev, reps, with_claim):
    """The 128^3 constant-coefficient workload: its 146 MB sliced matrix stays in the
    256 MB Infinity Cache across the iteration (the phases stream the vectors past it),
    so its SpMV figures are cache bandwidth, reported with bound "cache", not HBM."""
    prob = g.problem("cd3d_128")
    A = pk.CSR.from_host(prob.A, dev)
    b = torch.from_numpy(prob.b).to(dev)
    xs = torch.from_numpy(prob.xstar).to(dev)
    n, nnz = prob.A.n, prob.A.nnz
    t, info, x = timed_solve(pk, torch, A, b, reps, tol=1e-10, max_iter=10000)
    kern, used, itk = kernel_table(pk, torch, A, b, n, nnz, info, x, 16)
    forms, x64 = fp64_forms(pk, torch, A, b, xs, 1, plain=(t, info, x))
    forms.update(precision_forms(pk, torch, A, b, xs, x64, forms, 1))
    out = {"workload": "cd3d_128: 3D upwind convection-diffusion 128^3, v=(30,20,10), seed 1; n=%d nnz=%d"
                       % (n, nnz),
           "regime": "Infinity-Cache-resident matrix: SpMV GB/s are cache bandwidth, not HBM",
           "seconds": t, "iterations": info["iterations"], "true_relres": info["true_relres"],
           "us_per_iteration": t / max(info["iterations"], 1) * 1e6,
           "kernels_in_solve": kern, "iteration_kernel_us": itk,
           "spmv_roofline": {"bound": "cache", "achieved": kern["spmv_seq"]["GBs"], "unit": "GB/s",
                             "note": "above the HBM copy ceiling because the matrix is served by the "
                                     "Infinity Cache; not an HBM fraction"},
           "forms": forms}
    if with_claim:
        out["exact_vs_plain_dots"] = claim_leg(pk, torch, A, b, n)
    log("cd3d_128:", json.dumps({k: v for k, v in out.items() if k != "exact_vs_plain_dots"}))
    return out


def micro_kernels(pk, torch, g, A, n, nnz, dev, reps):
    """HIP events around every launch on the launch stream: the SpMV kernel shapes on a
    cold cache (bytes: 12 per nonzero + 20 per row) and the standalone exact dot."""
    kern = {}
    S = pk.SlicedCSR(A)
    shapes = [("spmv_seq_cold", pk.SPMV_SEQ, None), ("spmv_vector_cold", pk.SPMV_VECTOR, None),
              ("spmv_wave_cold", pk.SPMV_WAVE, None)]
    if S.built:
        shapes.insert(0, ("spmv_seq_sliced_cold", pk.SPMV_SEQ, S))
    for name, kind, sl in shapes:
        dt, gbs = spmv_cold(pk, torch, A, min(reps, 10), kind, sl)
        kern[name] = {"us": dt * 1e6, "bytes": 12 * nnz + 20 * n, "GBs": gbs}   # 32-bit columns
    del S
    # standalone exact dot, rotating over buffers larger than the cache: uniform
    # U[-1, 1] at 2^20, 2^24, 2^26; wide exponents (+-1000) and exactly cancelling
    # (ill-conditioned) inputs at 2^24
    cases = [("uniform", 1 << 20), ("uniform", 1 << 24), ("uniform", 1 << 26),
             ("wide_exponent", 1 << 24), ("ill_conditioned", 1 << 24)]
    for fam, ne in cases:
        nbuf = max(2, int((768 << 20) // (16 * ne)))

        def vecs(i):
            if fam == "uniform":
                return (np.random.default_rng(10 + i).uniform(-1, 1, ne),
                        np.random.default_rng(20 + i).uniform(-1, 1, ne))
            if fam == "wide_exponent":
                return g.wide_exponent_vec(ne, 10 + i), g.wide_exponent_vec(ne, 20 + i, -20, 20)
            return g.cancelling_vec(ne, 10 + i), np.ones(ne)
        bufs = [tuple(torch.from_numpy(v).to(dev) for v in vecs(i)) for i in range(nbuf)]
        o1 = torch.empty(1, dtype=torch.float64, device=dev)
        wse = torch.empty(pk.lib().exdot_workspace_bytes(ne), dtype=torch.uint8, device=dev)
        cnt = [0]

        def f():
            xa, ya = bufs[cnt[0] % nbuf]
            cnt[0] += 1
            pk.exdot(xa, ya, o1, wse)
        dt = time_launches(f, reps, torch)
        key = f"exdot_2^{ne.bit_length() - 1}" + ("" if fam == "uniform" else f"_{fam}")
        kern[key] = {"us": dt * 1e6, "bytes": 16 * ne, "GBs": 16 * ne / dt / 1e9}
        del bufs
    # calibration of what streaming reaches on this part (torch's own element-wise kernels,
    # not this library's): a 1 GiB copy (read + write) and c = a + b over 1 GiB vectors
    # (two reads, one write), rotating over two sets so that nothing is cache-resident
    ne = 1 << 27
    sets = [[torch.empty(ne, dtype=torch.float64, device=dev).fill_(1.0) for _ in range(3)] for _ in range(2)]
    cnt = [0]

    def copy():
        a, b, _ = sets[cnt[0] % 2]
        cnt[0] += 1
        b.copy_(a)

    def add():
        a, b, c = sets[cnt[0] % 2]
        cnt[0] += 1
        torch.add(a, b, out=c)
    for key, fn, nb in (("stream_copy_1GiB", copy, 16 * ne), ("stream_add_1GiB", add, 24 * ne)):
        dt = time_launches(fn, min(reps, 10), torch)
        kern[key] = {"us": dt * 1e6, "bytes": nb, "GBs": nb / dt / 1e9, "kernel": "torch element-wise"}
    del sets
    for k, v in kern.items():
        v["frac_of_peak"] = v["GBs"] / HBM_PEAK_GBS
    log("micro kernels:", json.dumps(kern))
    return kern


def cpu_baseline(prob, gi):
    """The C oracle (exact dots, OpenMP) on the headline workload: a bounded sample of
    iterations (about 20 s of CPU work) with all threads and with one, each extrapolated
    per iteration to the GPU's iteration count gi."""
    from oracle import ctier
    host_cpus = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    res = {}
    all_threads = ctier.num_threads()
    for label, nt, budget in (("all", all_threads, 20.0), ("one", 1, 15.0)):
        ctier.set_threads(nt)
        t = time.perf_counter()
        ctier.pbicgstab(prob.A, prob.b, tol=1e-10, max_iter=0)
        t_init = time.perf_counter() - t
        t = time.perf_counter()
        ctier.pbicgstab(prob.A, prob.b, tol=1e-10, max_iter=2)
        per_it = max(time.perf_counter() - t - t_init, 1e-9) / 2
        k = int(max(2, min(gi, 200, budget / per_it)))
        t = time.perf_counter()
        rk = ctier.pbicgstab(prob.A, prob.b, tol=1e-10, max_iter=k)
        tk = time.perf_counter() - t
        per_it = max(tk - t_init, 1e-9) / max(rk["iterations"], 1)
        est = t_init + gi * per_it
        res[label] = {"threads": nt, "iterations_timed": rk["iterations"], "seconds_timed": tk,
                      "seconds_per_iteration": per_it, "init_s": t_init, "extrapolated_solve_s": est,
                      "complete": rk["iterations"] == gi and rk["status"] == 0}
        log(f"cpu oracle ({nt} threads): {rk['iterations']} iterations in {tk:.2f}s, {per_it * 1e3:.1f} ms each")
    ctier.set_threads(all_threads)
    a = res["all"]
    return {"value": a["extrapolated_solve_s"], "unit": "s", "cores": a["threads"], "kind": "oracle",
            "sample": (f"C oracle p-BiCGStab (exact dots, OpenMP) on the headline workload: "
                       f"{a['iterations_timed']} of the GPU's {gi} iterations timed ({a['seconds_timed']:.1f} s, "
                       f"{a['threads']} threads), extrapolated per iteration to {gi} iterations"
                       + ("" if not a["complete"] else "; complete solve")),
            "extrapolated": not a["complete"],
            "one_thread": {"value": res["one"]["extrapolated_solve_s"], "cores": 1,
                           "iterations_timed": res["one"]["iterations_timed"],
                           "seconds_per_iteration": res["one"]["seconds_per_iteration"]},
            "host_cpus": host_cpus, "cpu_model": model, "runs": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--solve-only", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the headline workload's other forms and the micro-benchmarks (legs still run)")
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--legs", default="cd3d_128,claim,cd2d_64,learned,rand_1m",
                    help="comma list of extra legs: cd3d_128, claim (needs cd3d_128), cd2d_64, learned, "
                         "rand_1m (empty: none)")
    ap.add_argument("--epochs", type=int, default=30, help="learned-preconditioner training epochs")
    ap.add_argument("--traffic-run", action="store_true",
                    help="launch each measured kernel 10 times (for rocprofv3 --pmc runs) and exit")
    ap.add_argument("--workload", default=HEADLINE,
                    help="workload of --traffic-run, or of a --solve-only profiling run (cd3d_256_var, cd3d_128)")
    ap.add_argument("--infer-run", action="store_true",
                    help="launch the bf16 inference on the held-out 128^3 matrix 10 times (for rocprofv3 "
                         "counter runs) and exit")
    args = ap.parse_args()
    if args.workload != HEADLINE and not (args.traffic_run or args.solve_only):
        print(json.dumps({"error": "--workload other than the headline needs --traffic-run or --solve-only"}))
        sys.exit(2)
    if args.workload not in WORKLOAD_DESC:
        print(json.dumps({"error": "unknown workload %s (choices: %s)" % (args.workload, ", ".join(WORKLOAD_DESC))}))
        sys.exit(2)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: bench.py measures one GPU's throughput; "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2404_13216_amd as pk
    import synthgen as g

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if args.infer_run:
        infer_run(pk, torch, g, dev)
        return
    t0 = time.time()
    wl = args.workload
    prob = g.problem(wl)
    A = pk.CSR.from_host(prob.A, dev)
    b = torch.from_numpy(prob.b).to(dev)
    n, nnz = prob.A.n, prob.A.nnz
    log(f"workload {wl} n={n} nnz={nnz} built in {time.time() - t0:.1f}s")

    if args.traffic_run:
        traffic_run(pk, torch, A, b, n, nnz, dev)
        return

    solver = pk.Solver(A, tol=1e-10, max_iter=10000)
    x = torch.zeros(n, dtype=torch.float64, device=dev)

    def step():
        x.zero_()
        return solver.solve(b, x)

    for _ in range(args.warmup):
        _, info = step()
        log(f"warmup solve: {info['iterations']} iterations, status {info['status']}")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = []
    for k in range(args.steps):
        _, info = step()
        infos.append(info)
        log(f"step {k + 1}/{args.steps}: {info['iterations']} iterations")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sec = elapsed / args.steps
    info = infos[-1]
    assert all(i["status"] == pk.OK and i["iterations"] == info["iterations"] for i in infos), infos
    xs = torch.from_numpy(prob.xstar).to(dev)
    err_xstar = rel(torch, x, xs)
    log(f"p-BiCGStab: {sec * 1e3:.2f} ms/solve, {info['iterations']} iterations, "
        f"true relres {info['true_relres']:.3e}")
    kern, used, iter_kernels_us = kernel_table(pk, torch, A, b, n, nnz, info, x, solver.opts.batch)
    log("kernels in the solve:", json.dumps(kern))

    out = {
        "metric": "time to true rel. residual 1e-10 (plain FP64 p-BiCGStab, exact dots) + SpMV HBM GB/s",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[wl],
                   "n": n, "nnz": nnz, "tol": 1e-10, "x0": "0", "alg": "p-BiCGStab",
                   "dots": "exact (rounded once)",
                   "spmv": "row-sequential, " + layout_name(info)},
        "iterations": info["iterations"],
        "true_relres": info["true_relres"],
        "rel_err_vs_xstar": err_xstar,
        "us_per_iteration": sec / max(info["iterations"], 1) * 1e6,
        "kernels_in_solve": kern,
        "iteration_kernel_us": iter_kernels_us,
    }
    # dominant kernel of the iteration: the SpMV (two launches per iteration)
    traffic = None
    tf = TRAFFIC_FILES[wl]
    if os.path.exists(tf):
        txt = open(tf).read()
        blob = txt[txt.index("```json") + 7: txt.index("```", txt.index("```json") + 7)]
        tr = json.loads(blob)
        if tr.get("source_hash") == kernel_source_hash() and "spmv_seq" in tr.get("kernels", {}):
            ks = tr["kernels"]
            traffic = (ks["spmv_seq"]["bytes_per_launch"] + ks.get("spmv_aw", ks["spmv_seq"])["bytes_per_launch"]) / 2
    sp = kern["spmv_seq"]
    out["roofline"] = {"kernel": "spmv_seq", "bound": "hbm" if wl == HEADLINE else "cache", "achieved": sp["GBs"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sp["GBs"] / HBM_PEAK_GBS,
                       "traffic": traffic, "algorithmic_bytes_per_launch": sp["bytes"],
                       "algorithmic_bytes": "12 per nonzero + 20 per row",
                       "layout_bytes_per_launch": sp["layout_bytes"], "layout_GBs": sp["layout_GBs"],
                       "avg_launch_us": sp["us"], "launches": sp["launches"],
                       "timing": "HIP events stamped by the kernel dispatches of iterations 1..%d of a solve "
                                 "identical to the timed ones" % used}

    if not args.solve_only:
        if not args.no_forms:
            forms, x64 = fp64_forms(pk, torch, A, b, xs, 1, plain=(sec, info, x))
            forms.update(precision_forms(pk, torch, A, b, xs, x64, forms, 1))
            out["forms"] = forms
            log("forms:", json.dumps(forms))
            out["micro_kernels"] = micro_kernels(pk, torch, g, A, n, nnz, dev, args.reps)
        # further legs run after the headline tables, so that they do not disturb them
        legs = [l for l in args.legs.split(",") if l]
        if "cd3d_128" in legs:
            out["cd3d_128"] = resident_leg(pk, torch, g, dev, 3, "claim" in legs)
        if "cd2d_64" in legs:
            out["cd2d_64"] = small_leg(pk, torch, g, dev)
        if "learned" in legs:
            out["learned_m"] = learned_leg(pk, torch, g, dev, 1, args.epochs)
        if "rand_1m" in legs:
            out.setdefault("other_workloads", {})["rand_1m"] = config_leg(pk, torch, g, dev, "rand_1m", 1)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, info["iterations"])
        log("cpu baseline:", json.dumps(out["cpu_baseline"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
