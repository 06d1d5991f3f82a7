/*
 * pbicgstab.h -- C-ABI of the MI355X (gfx950) exact-reduction pipelined BiCGStab library
 * (libpbicgstab.so).
 *
 * The library solves A x = b for a square, unsymmetric sparse A given in CSR form,
 * from b and x0, with the pipelined BiCGStab of Cools and Vanroose (paper: Algorithm 2)
 * or van der Vorst's BiCGStab (paper: Algorithm 1).  Every inner product of the FP64
 * solvers is accumulated exactly and rounded once to FP64, ExBLAS-style (paper,
 * Section 2, the paragraph on reproducibility of the pure-MPI solver): results do not
 * depend on launch shape, operation order or reduction tree.
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE pointers unless the comment says (host).
 *  - `stream` is a hipStream_t passed as void*; every call is stream-ordered.
 *    Only pbicgstab_solve synchronises (it polls a small status block between
 *    batches of iterations).  No call allocates device memory: the caller owns every
 *    buffer, including the workspace `ws` of `ws_bytes` bytes (256-byte aligned).
 *  - CSR: int32 row_ptr[n+1], int32 col_idx[nnz] (column indices in [0, n), sorted
 *    ascending within each row; range checks are the caller's responsibility),
 *    values FP64 (or FP32 where stated).  nnz < 2^31.
 *  - Return value: PBCG_OK (0), a positive informative status (solve only: the
 *    current iterate is returned in x and `info` is filled), or a negative error.
 *    Argument errors are detected on the host before anything is launched.
 *  - Calls that share a workspace must not overlap in time (different streams with
 *    different workspaces are independent).
 */
#ifndef PBICGSTAB_H
#define PBICGSTAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PBCG_OK = 0,
    PBCG_NOT_CONVERGED = 1,   /* max_iter reached before the true residual met tol       */
    PBCG_BREAKDOWN = 2,       /* a zero denominator (r_hat,w0), (y,y) with q != 0, omega,
                                 rho or the alpha denominator                                */
    PBCG_STAGNATED = 3,       /* 30 failed true-residual tests in a row without a new
                                 smallest true residual: the recursive residual no longer
                                 describes x (tolerance below what the recurrences
                                 sustain); x is the best tested iterate                  */
    PBCG_ERR_INVALID = -1,    /* bad argument (null pointer, n < 0, nnz mismatch, ...)     */
    PBCG_ERR_HIP = -2,        /* a HIP runtime call failed                                  */
    PBCG_ERR_NONFINITE = -3,  /* NaN/Inf in b or in a recurrence scalar                     */
    PBCG_ERR_WORKSPACE = -4   /* ws == NULL or ws_bytes below the required size             */
} pbcg_status;

typedef enum { PBCG_F64 = 0, PBCG_F32 = 1 } pbcg_dtype;
typedef enum { PBCG_ALG_PBICGSTAB = 0, PBCG_ALG_BICGSTAB = 1 } pbcg_alg;
/* FP64: everything FP64 (exact dots).  FP32_IR: FP64 refinement around an FP32
 * p-BiCGStab (FP32 values, vectors and scalars; see pbicgstab_solve).  FP32_MATRIX: FP64
 * p-BiCGStab (FP64 vectors, FP64 accumulation, exact dots) whose iterations apply A's values
 * rounded to FP32 -- half the value bytes of every SpMV -- with residual replacement
 * against the FP64 A every rr_period iterations (default 50): r = b - A x, and w, t, s, z,
 * v recomputed with the FP32 values; the true residual (FP64 A) decides convergence. */
typedef enum { PBCG_PREC_FP64 = 0, PBCG_PREC_FP32_IR = 1, PBCG_PREC_FP32_MATRIX = 2 } pbcg_prec;

/* SpMV kernel shape.  SEQ sums every row left to right in storage order (the order of
 * the plain definition of A.x, so results are reproducible bit for bit by a sequential
 * CPU loop); VECTOR uses L = 2..32 lanes per row (L from the mean row length) and
 * WAVE one 64-lane wavefront per row, both with a fixed tree order per matrix. */
typedef enum { PBCG_SPMV_SEQ = 0, PBCG_SPMV_VECTOR = 1, PBCG_SPMV_WAVE = 2 } pbcg_spmv_kind;

/* Inner products of the p-BiCGStab recurrences.  EXACT: accumulated exactly and rounded
 * once (paper, Section 2, the ExBLAS paragraph).  PLAIN: ordinary FP64 products and sums
 * in a fixed reduction tree -- the comparator for the paper's claim that exact dots keep
 * the recursive residual with the true one.  ||b||, the true residual and the (q, q)
 * test of a lucky breakdown stay exact in both. */
typedef enum { PBCG_DOTS_EXACT = 0, PBCG_DOTS_PLAIN = 1 } pbcg_dots;

/* Matrix layout of the solver's row-sequential SpMVs.  AUTO: the offset form when the
 * rows of every 256-row slice draw their columns from at most 8 offsets col - row
 * (banded and stencil matrices): per slice the offsets, per row a mask byte of the
 * offsets it has and one value slot per offset (0 where it has none), no column entries
 * and no row pointers read; its slots may exceed nnz by at most nnz/8 + 256.  Otherwise
 * as SLICED.  SLICED: the sliced layout of csr_slice when its padding stays within
 * nnz/8 + 256 entries; the copy stores each column entry as a 16-bit residual
 * col - row - base, with one 32-bit base per slice and entry position (the smallest
 * col - row there), when every residual fits (2 bytes per entry less); otherwise it
 * keeps CSR.  SORTED: a row-sorted copy instead (when its padding fits the same bound):
 * slices of 64 rows (one wavefront), the rows of every window of 4096 consecutive rows
 * ordered by decreasing length so that each slice holds rows of nearly equal length,
 * with a permutation back to the row order (4 bytes per row).  CSR: never copied.  All
 * give bit-identical results: every row is still summed left to right in storage order
 * by one lane. */
typedef enum {
    PBCG_LAYOUT_AUTO = 0,
    PBCG_LAYOUT_CSR = 1,
    PBCG_LAYOUT_SORTED = 2,
    PBCG_LAYOUT_SLICED = 3
} pbcg_layout;

/* Square CSR matrix.  `val` points to nnz values of type `val_type`. */
typedef struct {
    int32_t n;
    int32_t val_type;          /* pbcg_dtype */
    int64_t nnz;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const void* val;
} pbcg_csr;

/* Solver options (host struct). */
typedef struct {
    double tol;                /* stop when the TRUE relative residual ||b-Ax||/||b|| <= tol */
    int32_t max_iter;          /* iterations (FP64 solve) / FP32 iterations in total (IR)    */
    int32_t alg;               /* pbcg_alg                                                    */
    int32_t prec;              /* pbcg_prec                                                   */
    int32_t max_outer;         /* FP32-IR: reliable updates before the FP64 finish (60 if 0)  */
    double inner_tol;          /* FP32-IR: update threshold -- the FP32 iterations stop when
                                  their residual dropped by this factor (default 0.1 if 0)   */
    const pbcg_csr* M;         /* right preconditioner on the same n (NULL = none): the
                                  solver runs on A.M and returns x = M y                      */
    int32_t fallback;          /* with M: on breakdown / non-finite / stall restart the
                                  unpreconditioned solver from the better iterate             */
    int32_t history_len;       /* entries available in `history`                              */
    double* history;           /* optional device buffer: recursive ||r_i||/||b|| per iteration */
    double* r_out;             /* optional device n-vector: the final recursive residual     */
    int32_t batch;             /* iterations enqueued between status polls (default 16)      */
    int32_t stall_window;      /* with M + fallback: iterations without halving the recursive
                                  residual that count as a stall (default 200)               */
    int32_t spmv_kind;         /* pbcg_spmv_kind used for every A.v of the solve (default SEQ) */
    int32_t trace;             /* nonzero: one line per FP32-IR reliable update on stderr     */
    int32_t dots;              /* pbcg_dots (FP64 p-BiCGStab without M; default EXACT)         */
    int32_t rr_period;         /* > 0: residual replacement every rr_period iterations (paper,
                                  the p-BiCGStabRR variant): r = b - A x, w = A r, t = A w,
                                  s = A p, z = A s, v = A z; scalars kept.  FP64 p-BiCGStab
                                  without M only.  0: none                                    */
    int32_t true_every;        /* > 0 with true_history: after every true_every-th completed
                                  iteration i that the solve continues from, the true relative
                                  residual ||b - A x_i||/||b|| (exact dot) is written to
                                  true_history[i / true_every - 1] (FP64 p-BiCGStab without
                                  M; the iterates are not affected) -- the recursive / true
                                  residual gap                                                */
    int32_t true_history_len;  /* entries available in true_history                        */
    double* true_history;      /* optional device buffer                                     */
    int32_t layout;            /* pbcg_layout (default AUTO; SEQ SpMV kind only)              */
    int32_t kernel_events_len; /* entries of kernel_events (a multiple of 8; 0: none)          */
    void* const* kernel_events;/* optional host array of hipEvent_t, created by the caller
                                  with timing enabled (measurement only).  FP64 p-BiCGStab
                                  with exact dots, no M and the row-sequential SpMV (the
                                  default kind): the four kernels of iteration
                                  j = 1 .. kernel_events_len/8 (phase A, v = A z, phase B,
                                  t = A w) are launched with hipExtLaunchKernel, which stamps
                                  events [8(j-1) + 2k] and [8(j-1) + 2k + 1] with kernel k's
                                  start and end; events of iterations that do not run keep
                                  their previous state.  Results are unaffected.            */
    int32_t exact_rows;        /* exactly rounded SpMV rows (the reproducible-reduction idea
                                  of the paper's Section 2 applied to A x; FP64 p-BiCGStab
                                  without M): 0 off; 1 every b - A x (r0, the true residual,
                                  residual replacement, true-residual history) has each row
                                  b_i - sum_k a_ik x_k formed exactly and rounded once;
                                  2 as 1, and every A v of the iteration has exactly rounded
                                  rows too (csr_spmv_exact), so no result depends on a
                                  summation order.  Slower per SpMV (csr_spmv_exact).       */
} pbcg_opts;

/* Result summary (host struct). */
typedef struct {
    int32_t status;
    int32_t iterations;        /* completed loop bodies (FP32-IR: total inner iterations)   */
    int32_t outer_iterations;  /* FP32-IR refinement steps                                   */
    int32_t true_checks;       /* true-residual evaluations                                  */
    int32_t fell_back;         /* 1 if the preconditioned solve fell back                    */
    int32_t sliced;            /* bit 0: A, bit 1: M ran on a sliced copy (layout AUTO);
                                  bit 2: A's, bit 3: M's copy holds 16-bit column residuals;
                                  bit 4: A's, bit 5: M's copy is the row-sorted one;
                                  bit 6: A's, bit 7: M's copy is the offset form           */
    double true_relres;        /* ||b - A x|| / ||b|| of the returned x (exact dots)         */
    double rec_relres;         /* last recursive ||r|| / ||b||                               */
    double seconds;            /* host wall time of the call                                 */
    int64_t sliced_entries;    /* entries (value slots) of A's sliced copy; 0: A ran on CSR  */
} pbcg_info;

/* Device vectors of one p-BiCGStab iteration (for the phase entry points). */
typedef struct {
    double *x, *r, *rhat, *w, *t, *p, *s, *z, *q, *y, *v;
} pbcg_vectors;

/* ---------------------------------------------------------------------------------
 * Sparse matrix-vector product y = A x (paper: the products A p_i, A q_i, A z_i,
 * A w_i of Algorithms 1 and 2).  A: FP64 or FP32 values; x, y: FP64; FP64 accumulation
 * with every row summed left to right in storage order (PBCG_SPMV_SEQ).  y must not
 * alias x.
 */
int csr_spmv(const pbcg_csr* A, const double* x, double* y, void* stream);

/* y = A x with every row summed exactly and rounded once to nearest even (the exact
 * dot's definition applied to each row: exact zero gives +0, NaN / inf as in exdot), so
 * the result depends on no summation order (paper, Section 2, the ExBLAS paragraph).
 * A: FP64 or FP32 values; x, y: FP64, y != x.  Short rows (mean length <= 12) are summed
 * by one lane each in a register window when their terms span a few 32-bit chunks; other
 * rows by 16 lanes into an LDS long accumulator.  About 3-4x the time of csr_spmv. */
int csr_spmv_exact(const pbcg_csr* A, const double* x, double* y, void* stream);

/* Same with an explicit kernel shape (pbcg_spmv_kind). */
int csr_spmv_config(const pbcg_csr* A, const double* x, double* y, int32_t kind, void* stream);

/* FP32 y = A x with FP32 values and vectors (the refinement's FP32 operator).  Every
 * row is accumulated in FP32 in storage order with the compensated algorithm Dot2 of
 * Ogita, Rump and Oishi (2005): TwoProduct by fused multiply-add, TwoSum (Knuth), the
 * errors summed into a compensation term; y_i = fl(s + c) is as accurate as a sum in
 * twice the working precision, rounded once.  y must not alias x. */
int csr_spmv_f32(const pbcg_csr* A32, const float* x, float* y, void* stream);

/* Jacobi preconditioner values (the diagonal right preconditioner M = diag(1/a_ii)
 * used beside the learned one): m_out[i] = 1/a_ii, the FP64 reciprocal rounded once
 * to m_type (PBCG_F64 or PBCG_F32).  A must hold FP64 values; a row without a stored
 * diagonal entry gets 1/0 = +inf.  m_out: n device values of m_type. */
int csr_jacobi(const pbcg_csr* A, void* m_out, int32_t m_type, void* stream);

/* ---------------------------------------------------------------------------------
 * Sliced copy of a CSR matrix for the row-sequential SpMV (the layout of this library,
 * not of the paper; the products are those of csr_spmv, the paper's A p_i, A q_i ... of
 * Algorithms 1 and 2).  Slice c holds rows 256c .. 256c+255 column-major: entry k of row
 * 256c + t sits at slice_off[c] + 256 k + t, and every slice is padded to its longest
 * row (padding: column 0, value 0, never used in arithmetic).  One lane per row walks
 * its row in storage order, so csr_spmv_sliced and csr_spmv return the same bits.
 * Pays off for matrices of near-uniform row length (stencils); the solver makes and uses
 * one by itself (pbcg_opts.layout).
 */
typedef struct {
    int64_t entries;           /* padded entry count (also set when too large to build)     */
    const int64_t* slice_off;  /* [ceil(n/256) + 1] entry offsets; NULL: not built          */
    const int32_t* col;        /* [entries] column indices                                  */
    const void* val;           /* [entries] values, A's val_type                            */
} pbcg_sliced;

/* Workspace csr_slice needs for an n x n matrix with nnz entries. */
size_t csr_slice_workspace_bytes(int32_t n, int64_t nnz);

/* Builds the sliced copy of A inside `ws` (device, 256-byte aligned, at least
 * csr_slice_workspace_bytes(n, nnz)); S (host) receives pointers into ws, valid while ws
 * is.  When the padding exceeds nnz/8 + 256 entries nothing is copied, S->slice_off is
 * NULL and S->entries holds the padded count: keep using CSR.  Synchronises `stream`
 * (the padded size is read back).  Errors: PBCG_ERR_INVALID (bad A or S),
 * PBCG_ERR_WORKSPACE, PBCG_ERR_HIP. */
int csr_slice(const pbcg_csr* A, pbcg_sliced* S, void* ws, size_t ws_bytes, void* stream);

/* y = A x as csr_spmv (bit-identical), reading the sliced copy S made by csr_slice from
 * this A.  x, y: FP64 device vectors, x != y.  PBCG_ERR_INVALID if S was not built. */
int csr_spmv_sliced(const pbcg_csr* A, const pbcg_sliced* S, const double* x, double* y, void* stream);

/* y = A x as csr_spmv_f32 (Dot2-compensated FP32, bit-identical), reading the sliced
 * copy S of the FP32 matrix A. */
int csr_spmv_f32_sliced(const pbcg_csr* A, const pbcg_sliced* S, const float* x, float* y, void* stream);

/* ---------------------------------------------------------------------------------
 * Exact dot product (paper Section 2, ExBLAS paragraph): *out = RN_even(sum x_i y_i)
 * with the sum formed exactly -- bit-identical for every launch shape.  Exact zero
 * gives +0; |sum| >= 2^1024 - 2^970 gives +-inf; NaN input, inf*0 or both +inf and
 * -inf products give NaN; otherwise an inf product gives that inf.  n >= 0.
 * `out` is one device double.  Needs exdot_workspace_bytes(n) bytes of workspace.
 */
size_t exdot_workspace_bytes(int64_t n);
int exdot(int64_t n, const double* x, const double* y, double* out,
          void* ws, size_t ws_bytes, void* stream);

/* Same as exdot with an explicit launch shape (grid >= 1 blocks of `block` in
 * {64,128,256,512,1024} threads) and per-lane expansion length k in {2,3,4,6,8}.
 * The result is independent of all three.  Workspace: exdot_workspace_bytes(n) covers
 * grid <= 1024. */
int exdot_config(int64_t n, const double* x, const double* y, double* out,
                 int32_t grid, int32_t block, int32_t k,
                 void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Plain (not exact) dot product: the inner products of the FP32 solver inside the
 * refinement (dtype PBCG_F32: FP32 products and sums) and of the ordinary-dot
 * comparator (PBCG_F64).  Each product is rounded to dtype and the sum is formed in a
 * fixed reduction tree: per-lane sums over a grid-stride loop, a butterfly within each
 * 64-lane wavefront, the block's wavefronts in index order, then a 256-wide tree over the
 * block partials.  The order depends on n only (not on the stream or timing), so the
 * result is reproducible run to run; it is not the sequential order, and its error
 * obeys the classical bound |dot - sum x_i y_i| <= gamma_n sum |x_i y_i|,
 * gamma_n = n u / (1 - n u).  x, y: n device values of dtype; out: one device value of
 * dtype.  Workspace: plain_dot_workspace_bytes(n).
 */
size_t plain_dot_workspace_bytes(int64_t n);
int plain_dot(int64_t n, const void* x, const void* y, int32_t dtype, void* out,
              void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Allocation-free exact dot, for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same result as exdot, bit for bit, with the same kernels; the per-block
 * records live in a static device array of exdot_noalloc_scratch_bytes() bytes (about
 * 0.55 MB), one copy per GPU, held until the process ends.  The array's device address
 * is looked up once per device on the first call there, which must run with the
 * stream's device current (PBCG_ERR_INVALID otherwise).  No call allocates or frees
 * memory.  n <= EXDOT_NOALLOC_MAX_N (2^34, beyond any vector pair that fits the GPU);
 * a larger n returns PBCG_ERR_INVALID before anything is launched.  Every call on one
 * GPU uses the same array: calls that overlap in time on that GPU (different streams,
 * threads or processes sharing the device) race and may return wrong results --
 * serialise them.  Nothing in the array needs to start at zero (each launched block
 * rewrites its whole record before it is read).
 */
#define EXDOT_NOALLOC_MAX_N ((int64_t)1 << 34)
size_t exdot_noalloc_scratch_bytes(void);
int exdot_noalloc(int64_t n, const double* x, const double* y, double* out, void* stream);

/* ---------------------------------------------------------------------------------
 * One fused pass of p-BiCGStab (paper Algorithm 2).  `scal` is a device array
 * {alpha, beta, omega}.
 * Phase A: p = r + beta (p - omega s); s = w + beta (s - omega z); z = t + beta (z - omega v)
 *          (first != 0: p = r, s = w, z = t);  q = r - alpha s;  y = w - alpha z;
 *          dots_out[0..3] = (q,y), (y,y), (r_hat,s), (r_hat,z)   (exact, device).
 * Phase B: x = (x + alpha p) + omega q;  r = q - omega y;  w = y - omega (t - alpha v);
 *          dots_out[0..2] = (r_hat,r), (r_hat,w), (r,r)             (exact, device).
 * Every update is evaluated in this parenthesisation with separately rounded operations.
 * Workspace: pbcg_phase_workspace_bytes(n).
 */
size_t pbcg_phase_workspace_bytes(int32_t n);
int pbcg_phase_a(int32_t n, const pbcg_vectors* V, const double* scal, int32_t first,
                 double* dots_out, void* ws, size_t ws_bytes, void* stream);
int pbcg_phase_b(int32_t n, const pbcg_vectors* V, const double* scal,
                 double* dots_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Solve A x = b (paper: p-BiCGStab(A, b, x0), Algorithm 2; BiCGStab(A, b, x0),
 * Algorithm 1).  x holds x0 on entry and the returned iterate on exit.  Stopping: the
 * recursive residual sqrt((r,r))/||b|| is checked every iteration; when it is <= tol
 * the true residual ||b - A x||/||b|| is evaluated and the solve stops if it is <= tol.
 * After a failed test the next one comes 5 iterations later; 30 failed tests in a row
 * without a new smallest true residual end the solve with PBCG_STAGNATED and x set to
 * the iterate of the best failed test.
 * prec = PBCG_PREC_FP32_IR: FP64 iterative refinement around an FP32 p-BiCGStab (FP32
 * values, vectors and scalars, the compensated FP32 SpMV of csr_spmv_f32, plain FP32
 * dot products in a fixed reduction tree) with reliable updates.  The FP32 process
 * accumulates a correction d; when its residual has dropped by inner_tol (or it looks
 * converged, breaks down or stalls) x = x + nu d, the true residual b - A x and its
 * exact norm nu are formed in FP64, and the FP32 process continues from r / nu with its
 * search direction kept (the paper's residual replacement: w, t, s, z, v recomputed)
 * or, after a breakdown or stall, restarts.  An update that does not lower the true
 * residual below the best so far (FP32 has reached its accuracy floor, about
 * u32 cond(A)), max_outer updates or max_iter FP32 iterations end in FP64 p-BiCGStab
 * from the best iterate, with residual replacement every 50 iterations
 * (info->fell_back = 1).
 * `info` (host) may be NULL.  Workspace: pbicgstab_workspace_bytes(n, nnz, opts); with
 * layout AUTO, SLICED or SORTED it includes room for the solver's copies of A and M (12
 * bytes per entry, nnz + nnz/8 + 256 entries each, which also hold the offset form),
 * which every call rebuilds (one or two stream synchronisations each).
 */
size_t pbicgstab_workspace_bytes(int32_t n, int64_t nnz, const pbcg_opts* opts);
int pbicgstab_solve(const pbcg_csr* A, const double* b, double* x, const pbcg_opts* opts,
                    pbcg_info* info, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Learned sparse approximate inverse M on A's pattern (right preconditioner for
 * pbicgstab_solve via opts->M).  m_ij = ([i == j] + f(phi_ij)) / a_ii with f an MLP
 * 12 -> 64 -> 64 -> 1 (GELU, erf form) over 12 per-nonzero features phi_ij; with the
 * last layer zero M is Jacobi.  Parameters: 5057 FP32 values, flat layout
 * W1[64x12] row-major, b1[64], W2[64x64] row-major, b2[64], w3[64], b3.
 * A must have FP64 values and n, nnz > 0.  No call allocates device memory.
 */
int spai_param_count(void);
size_t spai_workspace_bytes(int32_t n, int64_t nnz, int32_t k);

/* Features (nnz x 12 FP32, row-major per nonzero), the row index of every nonzero
 * and diag[i] = a_ii (FP64, 0 if absent).  Column sums of |A| use exact fixed-point
 * integer accumulation (order independent). */
int spai_features(const pbcg_csr* A, float* feat, int32_t* rowidx, double* diag,
                  void* ws, size_t ws_bytes, void* stream);

/* FP32 MLP forward: f_out (nnz, may be NULL) and m_out (nnz) = M values. */
int spai_forward(int64_t nnz, const float* feat, const float* params, const int32_t* rowidx,
                 const int32_t* col_idx, const double* diag, float* f_out, float* m_out, void* stream);

/* bf16 inference with MFMA: weights and layer inputs rounded to bf16 (nearest even),
 * FP32 accumulation, GELU in FP32 by linear interpolation in a table of 4,096 intervals
 * (absolute error below 2e-6, before the bf16 rounding of the layer output), M values
 * stored FP32. */
int spai_infer_bf16(int64_t nnz, const float* feat, const float* params, const int32_t* rowidx,
                    const double* diag, float* m_out, void* stream);

/* One residual column of a probe block (the training objective's V holds residuals
 * r_i / ||r_i|| of a plain p-BiCGStab run on the training matrix):
 * out[i] = fp32(r_i / ||r||_2), ||r||_2 the square root of the exact dot (r, r) (rounded
 * once, as every inner product here); r = 0 gives a zero column.  r: n device doubles,
 * out: n device floats (e.g. a column of a column-major V).  Workspace:
 * spai_probe_column_workspace_bytes(n). */
size_t spai_probe_column_workspace_bytes(int32_t n);
int spai_probe_column(int32_t n, const double* r, float* out, void* ws, size_t ws_bytes, void* stream);

/* U = A V for a probe block V (n x k, column-major FP32); FP64 row sums stored FP32. */
int spai_probe_product(const pbcg_csr* A, const float* V, int32_t k, float* U, void* stream);

/* Loss L = ||M U - V||_F^2 / (k n) (M from the FP32 forward, written to m_tmp) and its
 * gradient with respect to the 5057 parameters; every reduction in a fixed order. */
int spai_loss_grad(const pbcg_csr* A, const float* feat, const int32_t* rowidx, const double* diag,
                   const float* params, const float* V, const float* U, int32_t k, float* m_tmp,
                   float* loss, float* grad, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma and Ba) on the parameters, t >= 1. */
int spai_adam(float* params, float* m, float* v, const float* grad, int32_t t, float lr,
              float b1, float b2, float eps, void* stream);

/* One training step on one matrix: spai_loss_grad then spai_adam, with the step's M
 * values and gradient kept in the workspace (spai_workspace_bytes(n, nnz, k)).
 * feat / rowidx / diag from spai_features; V, U = A V (spai_probe_product) n x k
 * column-major; adam_m, adam_v: 5057 device floats each (zero before step t = 1);
 * hyper (host): {lr, beta1, beta2, eps}; loss: one device float (this step's loss,
 * before the update). */
int spai_train_step(const pbcg_csr* A, const float* feat, const int32_t* rowidx, const double* diag,
                    const float* V, const float* U, int32_t k, float* params, float* adam_m, float* adam_v,
                    int32_t t, const float* hyper, float* loss, void* ws, size_t ws_bytes, void* stream);

/* Fill `opts` (host) with defaults: tol 1e-10, max_iter 10000, p-BiCGStab, FP64. */
void pbcg_default_opts(pbcg_opts* opts);

/* Human-readable name of a status code (static string). */
const char* pbcg_status_string(int status);

/* Library ABI version (bumped on any change of the structs above). */
int pbcg_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PBICGSTAB_H */
