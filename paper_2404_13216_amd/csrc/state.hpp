// Device-resident solver state shared by the kernels and the host driver.
#pragma once
#include <stdint.h>

namespace pbcg {

// halt reasons (bit set)
enum : int {
    R_CHECK = 1,        // recursive residual <= tol: host evaluates the true residual
    R_NONFINITE = 2,    // a non-finite recurrence scalar
    R_BREAKDOWN = 4,    // zero denominator
    R_MAXIT = 8,        // iteration limit reached
    R_YYZERO = 16,      // (y,y) == 0: host tests (q,q) for a lucky breakdown
    R_ZERO_RHS = 32,    // ||b|| == 0
    R_CONVERGED = 64,   // (inner FP32 solve) recursive tolerance met
    R_STALL = 128,      // recursive residual not halved over stall_window iterations
};

// FP64 solver scalars.  alpha, beta, omega are consecutive: kernels read them
// through a `const double* scal` = &alpha.
//
// Halting: finalize roles set `halt`; phase kernels skip when `halt` is set and then
// raise `halt_seen`; SpMV kernels of the iteration loop skip only on `halt_seen`.  An
// SpMV whose block 0 carries a finalize that halts therefore still completes all of its
// rows (a resumed solve needs its output), and SpMVs queued after a halt recompute
// nothing new (their inputs are frozen) or are skipped.
struct State {
    double alpha, beta, omega, rho;
    double rs, rz, qy, yy;
    double normb, rec, true_rel, tol;
    double rw, rr, last_dot, pad0;
    int32_t iter, max_iter, halt, reason;
    int32_t hist_len, true_checks, halt_seen, stall_window;
    int32_t check_it, pad_i;   // iteration of the last failed true-residual test (-1: none)
    double* hist;
    double* stall_hist;     // full per-iteration history for stall detection (or null)
};

// State of the FP32 iterations of the refinement solver.  rec = sqrt((r, r)) in units
// of the last reliable update's residual norm; tol: the update threshold on rec; lim:
// the rec below which the solve looks converged (tol ||b|| / nu).
struct FState {
    float alpha, beta, omega, rho;
    float rs, rz, pad0, rec;
    float tol, best, lim, pad2;      // best: smallest rec since the last update
    int32_t iter, max_iter, halt, reason;
    int32_t halt_seen, it_best, stall, fpad2;   // stall: iterations without a new best that stop
};

}  // namespace pbcg
