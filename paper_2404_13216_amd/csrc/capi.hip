// C-ABI of libpbicgstab.so: argument checks, workspace layout, kernel launches and
// the host driver of the solvers.  See include/pbicgstab.h for the contract.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/pbicgstab.h"
#include "kernels.hpp"
#include "exact_rows.hpp"

using namespace pbcg;

namespace {

constexpr int BLOCK = 256;
constexpr int DOT_BLOCK = 512;       // fused element-wise kernels with exact dots
constexpr int DOT_GRID_MAX = 1024;   // records available in a dot site
constexpr int DOT_GRID_DEFAULT = 256;
constexpr int IR_INNER_STALL = 100;   // FP32 iterations without a new minimum
constexpr int IR_MAX_UPDATES = 60;    // reliable updates before the FP64 finish
constexpr int IR_MAX_BAD = 1;         // updates that did not improve on the best before it
constexpr double IR_DELTA = 0.1;      // default update threshold (inner_tol)
constexpr int IR_FP64_FINISH = 10000; // iteration limit of the FP64 finish after stagnation
constexpr int IR_FINISH_RR = 50;      // residual replacement period of that finish
constexpr int IR_BATCH = 4;           // FP32 iterations enqueued between status polls (at most)
constexpr int KEXP = 3;              // expansion terms per lane in the solver kernels
constexpr int EXDOT_U = 4;           // elements per lane and trip of a single exact dot (2 loads each)
constexpr int EXDOT_BLOCK = 1024;    // threads per block of the standalone exact dot
constexpr int PHASE_U = 2;           // the same for the fused phases (7 or 8 loads each)
constexpr double INFINITY_CACHE_BYTES_D = 256.0 * 1024 * 1024;   // MI355X Infinity Cache
constexpr int FP32M_RR = 50;          // default replacement period of the FP32-matrix form

#define HIPCHK(expr)                              \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return PBCG_ERR_HIP; \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------- workspace carving
struct Carver {
    char* base;
    size_t off = 0;
    size_t limit;
    bool ok = true;
    explicit Carver(void* b, size_t lim) : base((char*)b), limit(lim) {}
    template <class T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = (T*)(base ? base + off : nullptr);
        off += count * sizeof(T);
        if (off > limit) ok = false;
        return p;
    }
};

size_t site_bytes(int grid_max) {
    return align_up((size_t)grid_max * 4 * sizeof(xd::RecHdr), 256) +
           align_up((size_t)grid_max * 4 * xd::NCH * sizeof(long long), 256) + 2 * 256;
}

xd::Site carve_site(Carver& c, int grid_max) {
    xd::Site s;
    s.hdr = c.take<xd::RecHdr>((size_t)grid_max * 4);
    s.dig = c.take<long long>((size_t)grid_max * 4 * xd::NCH);
    return s;
}

// blocks of DOT_BLOCK threads, >= 8 elements per lane, at most one block per CU
// grid of the plain (fixed-tree) dots: 8 elements per lane, at most 256 blocks (the tree's
// shape, which fixes the plain dots' rounding, follows from it)
int dot_grid(int64_t n) {
    int64_t g = (n + (int64_t)DOT_BLOCK * 8 - 1) / ((int64_t)DOT_BLOCK * 8);
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, DOT_GRID_DEFAULT));
}

// grid of the fused phases and of the solver's other exact dots: one element per lane until
// 256 blocks are reached, so a small system spreads its rows over several compute units (8
// elements per lane put a 4,096-row system's phase on one block: 15.8 us for phase A); the
// exact dots' bits do not depend on the grid
int xdot_grid(int64_t n) {
    int64_t g = (n + (int64_t)DOT_BLOCK - 1) / (int64_t)DOT_BLOCK;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, DOT_GRID_DEFAULT));
}

// lanes per row from the mean row length (fixed per matrix -> fixed summation order)
int spmv_lanes(int32_t n, int64_t nnz) {
    double mean = n > 0 ? (double)nnz / (double)n : 1.0;
    int L = 2;
    while (L < mean && L < 64) L <<= 1;
    return L;
}

bool csr_ok(const pbcg_csr* A) {
    return A && A->n >= 0 && A->nnz >= 0 && A->nnz < (int64_t(1) << 31) &&
           (A->n == 0 || (A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val)))) &&
           (A->val_type == PBCG_F64 || A->val_type == PBCG_F32);
}

// A matrix as the launchers see it: the CSR arrays and, when one was built, a sliced
// copy with the same row order (read by the row-sequential kernels only).
struct SliceView {
    const int64_t* off = nullptr;
    const int32_t* col = nullptr;   // 32-bit columns, or 16-bit residuals when d16
    const void* val = nullptr;
    bool nt = false;    // matrix larger than the Infinity Cache: stream it (non-temporal loads)
    bool d16 = false;   // column entries are 16-bit residuals from a per-position base
    const int32_t* base = nullptr;  // per slice and position (d16)
    const int32_t* perm = nullptr;  // row-sorted copy (64-row slices): the row of each slot
    const uint8_t* mask = nullptr;  // offset form: per row, the slots it has
    const int32_t* ofs = nullptr;   // offset form: per slice, OFS_MAX offsets col - row
};

// the runtime layout of a sliced copy -> the kernels' compile-time layout flags
template <class F>
void with_slf(const SliceView& v, F&& f) {
    if (v.mask) {   // offset form: no column entries
        if (v.nt) f(std::integral_constant<int, SL_OFS | SL_NT>{});
        else f(std::integral_constant<int, SL_OFS>{});
        return;
    }
    if (v.perm) {   // row-sorted copies keep 32-bit columns
        if (v.nt) f(std::integral_constant<int, SL_PERM | SL_NT>{});
        else f(std::integral_constant<int, SL_PERM>{});
        return;
    }
    switch ((v.nt ? SL_NT : 0) | (v.d16 ? SL_D16 : 0)) {
        case 0: f(std::integral_constant<int, 0>{}); break;
        case SL_NT: f(std::integral_constant<int, SL_NT>{}); break;
        case SL_D16: f(std::integral_constant<int, SL_D16>{}); break;
        default: f(std::integral_constant<int, SL_NT | SL_D16>{}); break;
    }
}

struct Mat {
    const pbcg_csr* csr = nullptr;
    SliceView sl{};
    Mat() = default;
    Mat(const pbcg_csr* c) : csr(c) {}
    Mat(const pbcg_csr* c, SliceView v) : csr(c), sl(v) {}
    const pbcg_csr* operator->() const { return csr; }
    explicit operator bool() const { return csr != nullptr; }
};

template <class VT>
Sliced<VT> typed(const SliceView& v) {
    return Sliced<VT>{v.off, v.col, (const VT*)v.val, v.base, v.perm, v.mask, v.ofs};
}

// A sliced copy is kept when its padding is at most nnz/8 + 256 entries.
int64_t slice_cap(int64_t nnz) { return nnz + nnz / 8 + 256; }
int nslices(int32_t n) { return (n + 255) / 256; }
int nwslices(int32_t n) { return (n + WS_ROWS - 1) / WS_ROWS; }
// entries of a slice-offset array that serves both layouts (+ one scratch slot)
size_t slice_off_len(int32_t n) { return (size_t)std::max(nslices(n), nwslices(n)) + 2; }

// Builds the sliced copy of A (n > 0) into off[nslices + 2] (the last entry is scratch),
// col[cap], val[cap] (A's value type) and, with allow16, sbase[cap / 256 + 1].  With
// allow16 and every residual col - row - base[c][k] within 16 bits the column entries are
// stored as 16-bit residuals (*d16 = true).  Returns the padded entry count -- above cap
// nothing was filled and the caller keeps the CSR form -- or -1 on a HIP error.
// Synchronises the stream once.
int64_t build_slices(const pbcg_csr* A, int64_t* off, int32_t* col, void* val, int32_t* sbase, int64_t cap,
                     hipStream_t s, bool allow16, bool* d16) {
    const int n = A->n, ns = nslices(n);
    *d16 = false;
    slice_clear_kernel<<<1, 1, 0, s>>>(off + ns + 1);
    slice_width_kernel<<<ns, 256, 0, s>>>(n, A->row_ptr, off);
    slice_scan_kernel<<<1, 1024, 0, s>>>(ns, off);
    if (allow16)
        slice_base_kernel<<<ns, 256, 0, s>>>(n, A->row_ptr, A->col_idx, off, cap, sbase,
                                             (unsigned long long*)(off + ns + 1));
    int64_t tm[2] = {0, 0};   // padded entries, residual-overflow flag
    if (hipMemcpyAsync(tm, off + ns, sizeof(tm), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    const int64_t total = tm[0];
    if (total > cap) return total;
    *d16 = allow16 && tm[1] == 0;
    auto fill = [&](auto vt, auto d) {
        using VT = decltype(vt);
        slice_fill_kernel<VT, decltype(d)::value><<<ns, 256, 0, s>>>(n, A->row_ptr, A->col_idx, (const VT*)A->val,
                                                                     off, sbase, col, (VT*)val);
    };
    if (A->val_type == PBCG_F64) {
        if (*d16) fill(double{}, std::true_type{});
        else fill(double{}, std::false_type{});
    } else {
        if (*d16) fill(float{}, std::true_type{});
        else fill(float{}, std::false_type{});
    }
    if (hipGetLastError() != hipSuccess) return -1;
    return total;
}

// Builds the row-sorted copy of A (n > 0): perm[n], off[nwslices + 2], col[cap], val[cap].
// Returns the padded entry count (above cap nothing was filled) or -1 on a HIP error.
// Synchronises the stream once.
int64_t build_wslices(const pbcg_csr* A, int32_t* perm, int64_t* off, int32_t* col, void* val, int64_t cap,
                      hipStream_t s) {
    const int n = A->n, nws = nwslices(n), nb = (n + 255) / 256;
    wslice_sort_kernel<<<(n + WSORT - 1) / WSORT, 1024, 0, s>>>(n, A->row_ptr, perm);
    wslice_width_kernel<<<nb, 256, 0, s>>>(n, nws, A->row_ptr, perm, off);
    slice_scan_kernel<<<1, 1024, 0, s>>>(nws, off);
    int64_t total = 0;
    if (hipMemcpyAsync(&total, off + nws, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    if (total > cap) return total;
    if (A->val_type == PBCG_F64)
        wslice_fill_kernel<double><<<nb, 256, 0, s>>>(n, nws, A->row_ptr, A->col_idx, (const double*)A->val, perm,
                                                      off, col, (double*)val);
    else
        wslice_fill_kernel<float><<<nb, 256, 0, s>>>(n, nws, A->row_ptr, A->col_idx, (const float*)A->val, perm,
                                                     off, col, (float*)val);
    if (hipGetLastError() != hipSuccess) return -1;
    return total;
}

// Builds the offset form of A (n > 0): off[nslices + 2] (the last entry is scratch),
// ofs[nslices * OFS_MAX], mask[nslices * 256] bytes, val[cap] (A's value type).  Returns the
// slot count (above cap nothing was filled), 0 when some slice has more than OFS_MAX
// offsets (nothing filled), or -1 on a HIP error.  Synchronises the stream once.
int64_t build_ofs(const pbcg_csr* A, int64_t* off, int32_t* ofs, uint8_t* mask, void* val, int64_t cap,
                  hipStream_t s) {
    const int n = A->n, ns = nslices(n);
    int* over = (int*)(off + ns + 1);
    slice_clear_kernel<<<1, 1, 0, s>>>(off + ns + 1);
    ofs_scan_kernel<<<ns, 256, 0, s>>>(n, A->row_ptr, A->col_idx, off, ofs, over);
    slice_scan_kernel<<<1, 1024, 0, s>>>(ns, off);
    int64_t tm[2] = {0, 0};   // slots, overflow flag
    if (hipMemcpyAsync(tm, off + ns, sizeof(tm), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    if (tm[1] != 0) return 0;
    if (tm[0] > cap) return tm[0];
    if (A->val_type == PBCG_F64)
        ofs_fill_kernel<double><<<ns, 256, 0, s>>>(n, A->row_ptr, A->col_idx, (const double*)A->val, off, ofs, mask,
                                                   (double*)val);
    else
        ofs_fill_kernel<float><<<ns, 256, 0, s>>>(n, A->row_ptr, A->col_idx, (const float*)A->val, off, ofs, mask,
                                                  (float*)val);
    if (hipGetLastError() != hipSuccess) return -1;
    return tm[0];
}

// ---------------------------------------------------------------- launchers
// Kernel timing for measurement: when a pair of events is pending, the next launch
// through klaunch goes through hipExtLaunchKernel, which stamps the events with that
// kernel's own start and end (no markers between kernels, so back-to-back launches keep
// their spacing).  Per host thread; consumed by one launch.
thread_local hipEvent_t g_kev[2] = {nullptr, nullptr};

template <typename... KArgs, typename... Args>
void klaunch(void (*k)(KArgs...), dim3 grid, dim3 block, size_t smem, hipStream_t s, Args... args) {
    if (g_kev[0]) {
        hipExtLaunchKernelGGL(k, grid, block, (std::uint32_t)smem, s, g_kev[0], g_kev[1], 0u, KArgs(args)...);
        g_kev[0] = g_kev[1] = nullptr;
    } else {
        k<<<grid, block, smem, s>>>(KArgs(args)...);
    }
}

constexpr int SEQ_WORKERS = 8 * 256;   // persistent SpMV blocks: 8 resident per CU (16 KB LDS each)
constexpr int EXACT_ROW_WORKERS = 8 * 256;  // exact-row SpMV blocks (17 KB LDS each)
constexpr int SLICE_WORKERS = 1 << 24; // sliced-copy SpMV: one block per slice (no LDS staging)

// kind: PBCG_SPMV_SEQ (rows summed left to right), PBCG_SPMV_VECTOR (L lanes per row
// from the mean row length, tree order), PBCG_SPMV_WAVE (one wavefront per row).
template <class VT, class XT, class AT, class Epi, class Fin = NoFin>
void launch_spmv_t(const Mat& A, const XT* x, Epi epi, const int* halt, hipStream_t s,
                   int kind = PBCG_SPMV_SEQ, Fin fin = Fin{}) {
    const int n = A->n;
    const VT* val = (const VT*)A->val;
    if (kind == PBCG_SPMV_SEQ) {
        const int workers = std::min((n + BLOCK - 1) / BLOCK, A.sl.off ? SLICE_WORKERS : SEQ_WORKERS);
        const int grid = workers + (Fin::D > 0 ? 1 : 0);
        if (grid > 0) {
            if (A.sl.off)
                with_slf(A.sl, [&](auto m) {
                    klaunch(spmv_seq_kernel<VT, XT, AT, Epi, Fin, false, true, decltype(m)::value>, grid, BLOCK, 0,
                            s, n, A->row_ptr, A->col_idx, val, x, epi, fin, halt, typed<VT>(A.sl));
                });
            else
                klaunch(spmv_seq_kernel<VT, XT, AT, Epi, Fin>, grid, BLOCK, 0, s,
                        n, A->row_ptr, A->col_idx, val, x, epi, fin, halt, Sliced<VT>{});
        }
        return;
    }
    if (n > 0) {
        const int L = kind == PBCG_SPMV_WAVE ? 64 : std::min(spmv_lanes(A->n, A->nnz), 32);
        const int rows = BLOCK / L;
        const int grid = (n + rows - 1) / rows;
#define SPMV_CASE(LL) \
    case LL: spmv_kernel<LL, VT, XT, AT, Epi><<<grid, BLOCK, 0, s>>>(n, A->row_ptr, A->col_idx, val, x, epi, halt); break;
        switch (L) {
            SPMV_CASE(2) SPMV_CASE(4) SPMV_CASE(8) SPMV_CASE(16) SPMV_CASE(32) SPMV_CASE(64)
        }
#undef SPMV_CASE
    }
    if constexpr (Fin::D > 0) fin_kernel<Fin><<<1, Fin::BLOCK, 0, s>>>(fin);
}

// FP64 accumulation, values FP64 or FP32, x FP64
template <class Epi, class Fin = NoFin>
void launch_spmv64(const Mat& A, const double* x, Epi epi, const int* halt, hipStream_t s,
                   int kind = PBCG_SPMV_SEQ, Fin fin = Fin{}) {
    if (A->val_type == PBCG_F64) launch_spmv_t<double, double, double>(A, x, epi, halt, s, kind, fin);
    else launch_spmv_t<float, double, double>(A, x, epi, halt, s, kind, fin);
}

// FP32 row-sequential SpMV with Dot2-compensated accumulation (the refinement's FP32
// operator; `fin` rides on block 0 as in launch_spmv_t)
template <class Epi, class Fin = NoFin>
void launch_spmv32c(const Mat& A, const float* x, Epi epi, const int* halt, hipStream_t s, Fin fin = Fin{}) {
    const int n = A->n;
    const int workers = std::min((n + BLOCK - 1) / BLOCK, A.sl.off ? SLICE_WORKERS : SEQ_WORKERS);
    const int grid = workers + (Fin::D > 0 ? 1 : 0);
    if (grid > 0) {
        if (A.sl.off)
            with_slf(A.sl, [&](auto m) {
                spmv_seq_kernel<float, float, float, Epi, Fin, true, true, decltype(m)::value><<<grid, BLOCK, 0, s>>>(
                    n, A->row_ptr, A->col_idx, (const float*)A->val, x, epi, fin, halt, typed<float>(A.sl));
            });
        else
            spmv_seq_kernel<float, float, float, Epi, Fin, true><<<grid, BLOCK, 0, s>>>(
                n, A->row_ptr, A->col_idx, (const float*)A->val, x, epi, fin, halt, Sliced<float>{});
    }
}

template <int D, class VT, class Epi>
void launch_spmv_dot_t(const Mat& A, const double* x, Epi epi, xd::Site site, const int* halt,
                       hipStream_t s, int kind) {
    const int n = A->n;
    const VT* val = (const VT*)A->val;
    if (kind == PBCG_SPMV_SEQ) {
        // persistent: up to 4 blocks per CU (one dot record each)
        int grid = std::max(1, std::min(DOT_GRID_MAX, (n + BLOCK - 1) / BLOCK));
        if (A.sl.off)
            with_slf(A.sl, [&](auto m) {
                spmv_seq_dot_kernel<D, KEXP, VT, Epi, true, decltype(m)::value><<<grid, BLOCK, 0, s>>>(
                    n, A->row_ptr, A->col_idx, val, x, epi, site, halt, typed<VT>(A.sl));
            });
        else
            spmv_seq_dot_kernel<D, KEXP, VT, Epi><<<grid, BLOCK, 0, s>>>(n, A->row_ptr, A->col_idx, val, x, epi,
                                                                          site, halt, Sliced<VT>{});
        fin_kernel<XFin<D, Epi>><<<1, XFin<D, Epi>::BLOCK, 0, s>>>(XFin<D, Epi>{epi, site, grid, halt});
        return;
    }
    const int L = kind == PBCG_SPMV_WAVE ? 64 : std::min(spmv_lanes(A->n, A->nnz), 32);
    const int rows = BLOCK / L;
    int grid = std::max(1, std::min(DOT_GRID_DEFAULT, (n + rows - 1) / rows));
#define SD_CASE(LL) \
    case LL: spmv_dot_kernel<LL, D, KEXP, VT, Epi><<<grid, BLOCK, 0, s>>>(n, A->row_ptr, A->col_idx, val, x, epi, site, halt); break;
    switch (L) {
        SD_CASE(2) SD_CASE(4) SD_CASE(8) SD_CASE(16) SD_CASE(32) SD_CASE(64)
    }
#undef SD_CASE
    fin_kernel<XFin<D, Epi>><<<1, XFin<D, Epi>::BLOCK, 0, s>>>(XFin<D, Epi>{epi, site, grid, halt});
}

template <int D, class Epi>
void launch_spmv_dot(const Mat& A, const double* x, Epi epi, xd::Site site, const int* halt,
                     hipStream_t s, int kind = PBCG_SPMV_SEQ) {
    if (A->val_type == PBCG_F64) launch_spmv_dot_t<D, double>(A, x, epi, site, halt, s, kind);
    else launch_spmv_dot_t<D, float>(A, x, epi, site, halt, s, kind);
}

// Whether the exact-row kernels try the one-lane-per-row register path first: rows of
// mean length up to 12 (stencils).  Longer rows leave most lanes of a wave waiting for its
// longest row, and the 16-lane LDS path is faster there.
inline bool exact_rows_fast(const pbcg_csr* A) { return (int64_t)A->nnz <= (int64_t)12 * A->n; }

// Exactly rounded rows (RESID: r = b - A x rounded once per row); persistent blocks of
// 256 threads, block 0 extra when it carries a finalize role.
template <bool RESID, class Epi, class Fin = NoFin>
void launch_spmv_exact(const Mat& A, const double* x, const double* b, Epi epi, const int* halt, hipStream_t s,
                       Fin fin = Fin{}) {
    const int n = A->n;
    const bool fast = exact_rows_fast(A.csr);
    const int rows = fast ? BLOCK : XR_ROWS;
    const int grid = std::min((n + rows - 1) / rows, EXACT_ROW_WORKERS) + (Fin::D > 0 ? 1 : 0);
    if (grid <= 0) return;
    auto go = [&](auto vt, auto f) {
        using VT = decltype(vt);
        constexpr bool F = decltype(f)::value;
        if (F && A.sl.mask)   // the register path reads the offset form when the solver has one
            klaunch(spmv_exact_kernel<VT, Epi, Fin, RESID, true, true>, grid, BLOCK, 0, s, n, A->row_ptr,
                    A->col_idx, (const VT*)A->val, x, b, epi, fin, halt, typed<VT>(A.sl));
        else
            klaunch(spmv_exact_kernel<VT, Epi, Fin, RESID, F>, grid, BLOCK, 0, s, n, A->row_ptr, A->col_idx,
                    (const VT*)A->val, x, b, epi, fin, halt, Sliced<VT>{});
    };
    if (A->val_type == PBCG_F64) {
        if (fast) go(double{}, std::true_type{});
        else go(double{}, std::false_type{});
    } else {
        if (fast) go(float{}, std::true_type{});
        else go(float{}, std::false_type{});
    }
}

template <int D, bool RESID, class Epi>
void launch_spmv_exact_dot(const Mat& A, const double* x, const double* b, Epi epi, xd::Site site,
                           const int* halt, hipStream_t s) {
    const int n = A->n;
    const bool fast = exact_rows_fast(A.csr);
    const int rows = fast ? BLOCK : XR_ROWS;
    const int grid = std::max(1, std::min(DOT_GRID_MAX, (n + rows - 1) / rows));
    auto go = [&](auto vt, auto f) {
        using VT = decltype(vt);
        constexpr bool F = decltype(f)::value;
        if (F && A.sl.mask)
            spmv_exact_dot_kernel<D, KEXP, VT, Epi, RESID, true, true><<<grid, BLOCK, 0, s>>>(
                n, A->row_ptr, A->col_idx, (const VT*)A->val, x, b, epi, site, halt, typed<VT>(A.sl));
        else
            spmv_exact_dot_kernel<D, KEXP, VT, Epi, RESID, F><<<grid, BLOCK, 0, s>>>(
                n, A->row_ptr, A->col_idx, (const VT*)A->val, x, b, epi, site, halt, Sliced<VT>{});
    };
    if (A->val_type == PBCG_F64) {
        if (fast) go(double{}, std::true_type{});
        else go(double{}, std::false_type{});
    } else {
        if (fast) go(float{}, std::true_type{});
        else go(float{}, std::false_type{});
    }
    fin_kernel<XFin<D, Epi>><<<1, XFin<D, Epi>::BLOCK, 0, s>>>(XFin<D, Epi>{epi, site, grid, halt});
}

// Producer only: returns the finalize role, to be run by fin_kernel or by block 0 of
// the next SpMV.
template <int D, int GM = DOT_GMAX, class Op>
XFin<D, Op, GM> launch_ew_dot_deferred(Op op, int64_t n, xd::Site site, const int* halt, hipStream_t s,
                                       int grid = 0, int block = DOT_BLOCK, int K = KEXP, int* seen = nullptr) {
    if (grid <= 0) grid = xdot_grid(n);
    grid = std::min(grid, GM);
    if constexpr (D == 1) {  // the standalone dot exposes the expansion length
#define EW_CASE(KK) \
    case KK: ew_dot_kernel<D, KK, Op, EXDOT_U, true><<<grid, block, 0, s>>>(op, n, site, halt, seen); break;
        switch (K) {
            EW_CASE(2) EW_CASE(3) EW_CASE(4) EW_CASE(6) EW_CASE(8)
            default: ew_dot_kernel<D, KEXP, Op, EXDOT_U, true><<<grid, block, 0, s>>>(op, n, site, halt, seen);
        }
#undef EW_CASE
    } else {
        klaunch(ew_dot_kernel<D, KEXP, Op, PHASE_U>, grid, block, 0, s, op, n, site, halt, seen);
    }
    return XFin<D, Op, GM>{op, site, grid, halt};
}

template <int D, class Op>
void launch_ew_dot(Op op, int64_t n, xd::Site site, const int* halt, hipStream_t s,
                   int grid = 0, int block = DOT_BLOCK, int K = KEXP) {
    XFin<D, Op> f = launch_ew_dot_deferred<D>(op, n, site, halt, s, grid, block, K);
    fin_kernel<XFin<D, Op>><<<1, XFin<D, Op>::BLOCK, 0, s>>>(f);
}

// plain dots in the fixed tree (T = float: the FP32 solver; double: ordinary FP64 dots)
template <int D, class T, class Op>
TFin<T, D, Op> launch_ew_fdot_deferred(Op op, int64_t n, TSite<T> site, const int* halt, hipStream_t s,
                                       int* seen = nullptr) {
    int grid = dot_grid(n);
    ew_fdot_kernel<T, D, Op><<<grid, DOT_BLOCK, 0, s>>>(op, n, site, halt, seen);
    return TFin<T, D, Op>{op, site, grid, halt};
}

template <int D, class T, class Op>
void launch_ew_fdot(Op op, int64_t n, TSite<T> site, const int* halt, hipStream_t s) {
    TFin<T, D, Op> f = launch_ew_fdot_deferred<D>(op, n, site, halt, s);
    fin_kernel<TFin<T, D, Op>><<<1, TFin<T, D, Op>::BLOCK, 0, s>>>(f);
}

template <class F>
void launch_ew(F f, int64_t n, const int* halt, hipStream_t s) {
    if (n <= 0) return;
    int64_t g = std::min<int64_t>((n + BLOCK - 1) / BLOCK, 4096);
    ew_kernel<F><<<(int)g, BLOCK, 0, s>>>(f, n, halt);
}

template <class F>
void launch_single(F f, hipStream_t s) {
    single_kernel<F><<<1, 64, 0, s>>>(f);
}

// ---------------------------------------------------------------- small device functors
struct FnZeroU32 {
    unsigned int* p; int count;
    __device__ void operator()() const { for (int i = 0; i < count; ++i) p[i] = 0u; }
};
struct FnCopy {
    double* dst; const double* src;
    __device__ void operator()(int64_t i) const { dst[i] = src[i]; }
};
struct FnCopy3 {
    double *a, *b, *c; const double* src;
    __device__ void operator()(int64_t i) const { double v = src[i]; a[i] = v; b[i] = v; if (c) c[i] = v; }
};
struct FnZero {
    double* dst;
    __device__ void operator()(int64_t i) const { dst[i] = 0.0; }
};
struct FnAxpyState {      // x = x + alpha p  (alpha from state)
    double* x; const double* p; const State* st;
    __device__ void operator()(int64_t i) const { x[i] = x[i] + st->alpha * p[i]; }
};
// (BiCGStab) q and p are the operands of the SpMV that follows: plain stores
template <bool NT>
struct FnQ {              // q = r - alpha s
    double* q; const double* r; const double* s; const double* scal;
    __device__ void operator()(int64_t i) const { q[i] = get<NT>(r, i) - scal[0] * get<NT>(s, i); }
};
template <bool NT>
struct FnPUpdate {        // p = r + beta (p - omega s), skipped before the first iteration
    double* p; const double* r; const double* s; const State* st;
    __device__ void operator()(int64_t i) const {
        if (st->iter == 0) return;
        p[i] = get<NT>(r, i) + st->beta * (get<NT, double>(p, i) - st->omega * get<NT>(s, i));
    }
};
struct FnCastScaled {     // r32 = fp32(r / nu)
    float* r32; const double* r; const State* st;
    __device__ void operator()(int64_t i) const { r32[i] = (float)(r[i] / st->last_dot); }
};
struct FnIRUpdate {       // x = x + nu * fp64(d)
    double* x; const float* d; const State* st;
    __device__ void operator()(int64_t i) const { x[i] = x[i] + st->last_dot * (double)d[i]; }
};
struct FnCastVal {
    float* dst; const double* src;
    __device__ void operator()(int64_t i) const { dst[i] = (float)src[i]; }
};
struct FnZeroF {
    float* dst;
    __device__ void operator()(int64_t i) const { dst[i] = 0.0f; }
};
struct FnFAxpyState {
    float* x; const float* p; const FState* st;
    __device__ void operator()(int64_t i) const { x[i] = x[i] + st->alpha * p[i]; }
};
struct FnInitState {
    State* st; double tol; int max_iter; double* hist; int hist_len; int stall_window; double* stall_hist;
    __device__ void operator()() const {
        State z;
        memset(&z, 0, sizeof(z));
        z.tol = tol; z.max_iter = max_iter; z.hist = hist; z.hist_len = hist_len;
        z.stall_window = stall_window; z.stall_hist = stall_hist;
        z.check_it = -1;
        *st = z;
    }
};
struct FnInitFState {
    FState* st; float tol; int max_iter; int stall;
    __device__ void operator()() const {
        FState z;
        memset(&z, 0, sizeof(z));
        z.tol = tol; z.max_iter = max_iter; z.stall = stall;
        z.best = __int_as_float(0x7f800000);   // +inf
        *st = z;
    }
};
struct FnSetFState {       // a reliable update: new convergence limit, stall window restarts
    FState* st; float lim;
    __device__ void operator()() const {
        st->lim = lim;
        st->best = __int_as_float(0x7f800000);   // +inf
        st->it_best = st->iter;
        st->halt = 0; st->reason = 0; st->halt_seen = 0;
    }
};
struct FnFIterPlus {       // (y, y) = 0: d = d + alpha p completed one more FP32 iteration
    FState* st;
    __device__ void operator()() const { st->iter += 1; }
};
struct FnScaleF {          // p = p * sigma (FP32)
    float* p; float sigma;
    __device__ void operator()(int64_t i) const { p[i] = p[i] * sigma; }
};
struct FnSetCheckIt {      // after a failed true-residual test at iteration it
    State* st; int it;
    __device__ void operator()() const { st->check_it = it; }
};
struct FnResume {          // clear halt flags (host decided to continue)
    State* st;
    __device__ void operator()() const { st->halt = 0; st->reason = 0; st->halt_seen = 0; }
};
struct FnSqrtLastDot {     // last_dot = sqrt(last_dot)
    State* st;
    __device__ void operator()() const { st->last_dot = sqrt(st->last_dot); }
};
struct FnIterPlus {        // lucky breakdown: one more completed iteration
    State* st;
    __device__ void operator()() const { st->iter += 1; st->rec = 0.0; }
};
struct FinLastDot {
    State* st;
    __device__ void operator()(const double* d) const { st->last_dot = d[0]; }
};

// pinned host mirror of the state for polling
struct Pinned {
    State* s = nullptr;
    FState* f = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ready = false;
    // Thread-storage objects of a thread are destroyed before any static object (the HIP
    // runtime's included), so the release below runs while the runtime is still up.
    ~Pinned() {
        if (!ready) return;
        for (int i = 0; i < 2; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        (void)hipHostFree(s);
    }
};
thread_local Pinned g_pin;

int pin_init() {
    if (g_pin.ready) return 0;
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(State) + 2 * sizeof(FState), hipHostMallocDefault) != hipSuccess) return -1;
    g_pin.s = (State*)p;
    g_pin.f = (FState*)((char*)p + 2 * sizeof(State));
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&g_pin.ev[i], hipEventDisableTiming) != hipSuccess) return -1;
    g_pin.ready = true;
    return 0;
}

}  // namespace

// ============================================================================ C-ABI
// Jacobi values 1/a_ii (FP64 reciprocal, then rounded once to the output type); the
// diagonal entry is found by binary search in the row's ascending columns.
template <class MT>
__global__ void __launch_bounds__(256) jacobi_kernel(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ val, MT* __restrict__ m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = rp[i], hi = rp[i + 1] - 1;
    double d = 0.0;
    while (lo <= hi) {
        const int mid = lo + ((hi - lo) >> 1);
        const int c = ci[mid];
        if (c == i) { d = val[mid]; break; }
        if (c < i) lo = mid + 1; else hi = mid - 1;
    }
    m[i] = (MT)(1.0 / d);
}

extern "C" {

int pbcg_abi_version(void) { return 8; }

const char* pbcg_status_string(int status) {
    switch (status) {
        case PBCG_OK: return "ok";
        case PBCG_NOT_CONVERGED: return "not converged";
        case PBCG_BREAKDOWN: return "breakdown";
        case PBCG_STAGNATED: return "stagnated";
        case PBCG_ERR_INVALID: return "invalid argument";
        case PBCG_ERR_HIP: return "HIP runtime error";
        case PBCG_ERR_NONFINITE: return "non-finite value";
        case PBCG_ERR_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

void pbcg_default_opts(pbcg_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->max_iter = 10000;
    o->alg = PBCG_ALG_PBICGSTAB;
    o->prec = PBCG_PREC_FP64;
    o->max_outer = IR_MAX_UPDATES;
    o->inner_tol = IR_DELTA;
    o->batch = 16;
    o->stall_window = 200;
}

int csr_spmv_config(const pbcg_csr* A, const double* x, double* y, int32_t kind, void* stream) {
    if (!csr_ok(A) || (A->n > 0 && (!x || !y))) return PBCG_ERR_INVALID;
    if (x == y && A->n > 0) return PBCG_ERR_INVALID;
    if (kind != PBCG_SPMV_SEQ && kind != PBCG_SPMV_VECTOR && kind != PBCG_SPMV_WAVE) return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    launch_spmv64(A, x, EpiStore<double>{y}, nullptr, s, kind);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int csr_spmv_exact(const pbcg_csr* A, const double* x, double* y, void* stream) {
    if (!csr_ok(A) || (A->n > 0 && (!x || !y))) return PBCG_ERR_INVALID;
    if (x == y && A->n > 0) return PBCG_ERR_INVALID;
    launch_spmv_exact<false>(A, x, nullptr, EpiStore<double>{y}, nullptr, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int csr_spmv(const pbcg_csr* A, const double* x, double* y, void* stream) {
    return csr_spmv_config(A, x, y, PBCG_SPMV_SEQ, stream);
}

int csr_spmv_f32(const pbcg_csr* A, const float* x, float* y, void* stream) {
    if (!csr_ok(A) || A->val_type != PBCG_F32 || (A->n > 0 && (!x || !y)) || (x == y && A->n > 0))
        return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    launch_spmv32c(A, x, EpiStore<float>{y}, nullptr, s);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

size_t csr_slice_workspace_bytes(int32_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    Carver c(nullptr, SIZE_MAX);
    c.take<int64_t>((size_t)nslices(n) + 2);
    c.take<int32_t>((size_t)slice_cap(nnz));
    c.take<double>((size_t)slice_cap(nnz));
    return c.off + 256;
}

int csr_slice(const pbcg_csr* A, pbcg_sliced* S, void* ws, size_t ws_bytes, void* stream) {
    if (!csr_ok(A) || !S) return PBCG_ERR_INVALID;
    std::memset(S, 0, sizeof(*S));
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < csr_slice_workspace_bytes(A->n, A->nnz))
        return PBCG_ERR_WORKSPACE;
    if (A->n == 0) return PBCG_OK;
    Carver c(ws, ws_bytes);
    int64_t* off = c.take<int64_t>((size_t)nslices(A->n) + 2);
    int32_t* col = c.take<int32_t>((size_t)slice_cap(A->nnz));
    void* val = c.take<double>((size_t)slice_cap(A->nnz));
    bool d16 = false;   // the public copy keeps 32-bit columns
    const int64_t total = build_slices(A, off, col, val, nullptr, slice_cap(A->nnz), (hipStream_t)stream, false,
                                       &d16);
    if (total < 0) return PBCG_ERR_HIP;
    S->entries = total;
    if (total <= slice_cap(A->nnz)) {
        S->slice_off = off;
        S->col = col;
        S->val = val;
    }
    return PBCG_OK;
}

int csr_spmv_sliced(const pbcg_csr* A, const pbcg_sliced* S, const double* x, double* y, void* stream) {
    if (!csr_ok(A) || !S || (A->n > 0 && (!x || !y || !S->slice_off || !S->col || !S->val)) ||
        (x == y && A->n > 0))
        return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    launch_spmv64(Mat(A, SliceView{S->slice_off, S->col, S->val}), x, EpiStore<double>{y}, nullptr, s);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int csr_spmv_f32_sliced(const pbcg_csr* A, const pbcg_sliced* S, const float* x, float* y, void* stream) {
    if (!csr_ok(A) || A->val_type != PBCG_F32 || !S ||
        (A->n > 0 && (!x || !y || !S->slice_off || !S->col || !S->val)) || (x == y && A->n > 0))
        return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    launch_spmv32c(Mat(A, SliceView{S->slice_off, S->col, S->val}), x, EpiStore<float>{y}, nullptr, s);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int csr_jacobi(const pbcg_csr* A, void* m_out, int32_t m_type, void* stream) {
    if (!csr_ok(A) || A->val_type != PBCG_F64 || (A->n > 0 && !m_out)) return PBCG_ERR_INVALID;
    if (m_type != PBCG_F64 && m_type != PBCG_F32) return PBCG_ERR_INVALID;
    if (A->n == 0) return PBCG_OK;
    hipStream_t s = (hipStream_t)stream;
    const int grid = (A->n + 255) / 256;
    const double* val = (const double*)A->val;
    if (m_type == PBCG_F64) jacobi_kernel<double><<<grid, 256, 0, s>>>(A->n, A->row_ptr, A->col_idx, val, (double*)m_out);
    else jacobi_kernel<float><<<grid, 256, 0, s>>>(A->n, A->row_ptr, A->col_idx, val, (float*)m_out);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

}  // extern "C"

namespace {
// The standalone exact dot: vectors together larger than the Infinity Cache stream past it
// (non-temporal loads); smaller ones keep plain loads (a caller may reuse them).
void exdot_launch(int64_t n, const double* x, const double* y, double* out, xd::Site site, hipStream_t s,
                  int grid, int block, int k) {
    if (16.0 * (double)n > INFINITY_CACHE_BYTES_D) {
        DotsOp<1, FinStore, true> op{};
        op.a[0] = x; op.b[0] = y;
        op.fin = FinStore{out, 1};
        launch_ew_dot<1>(op, n, site, nullptr, s, grid, block, k);
    } else {
        DotsOp<1, FinStore> op{};
        op.a[0] = x; op.b[0] = y;
        op.fin = FinStore{out, 1};
        launch_ew_dot<1>(op, n, site, nullptr, s, grid, block, k);
    }
}
}  // namespace

extern "C" {

size_t exdot_workspace_bytes(int64_t n) {
    (void)n;
    return site_bytes(DOT_GRID_MAX);
}

int exdot_config(int64_t n, const double* x, const double* y, double* out, int32_t grid, int32_t block,
                 int32_t k, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || !out || (n > 0 && (!x || !y))) return PBCG_ERR_INVALID;
    if (grid < 1 || grid > DOT_GRID_MAX) return PBCG_ERR_INVALID;
    if (!(block == 64 || block == 128 || block == 256 || block == 512 || block == 1024)) return PBCG_ERR_INVALID;
    if (!(k == 2 || k == 3 || k == 4 || k == 6 || k == 8)) return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < exdot_workspace_bytes(n)) return PBCG_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    xd::Site site = carve_site(c, DOT_GRID_MAX);
    exdot_launch(n, x, y, out, site, s, grid, block, k);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free exact dot
// The records of exdot_noalloc live in a file-scope device array (one copy per GPU, held
// until the process ends).  Host code never passes `scratch` itself to a kernel: its name
// is a host-side stand-in; the device address comes from hipGetSymbolAddress, taken once
// per device with that device current.
namespace {
constexpr int NOALLOC_GRID = 512;    // the largest grid exdot launches
constexpr size_t NOALLOC_HDR = (size_t)NOALLOC_GRID * sizeof(xd::RecHdr);
constexpr size_t NOALLOC_BYTES = NOALLOC_HDR + (size_t)NOALLOC_GRID * xd::NCH * sizeof(long long);
static_assert(NOALLOC_HDR % 256 == 0, "chunk records start 256-byte aligned");
constexpr int NOALLOC_MAX_DEV = 64;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

int scratch_address(hipStream_t s, void** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (s) {
        int sdev = -1;
        HIPCHK(hipStreamGetDevice(s, &sdev));
        if (sdev != dev) return PBCG_ERR_INVALID;   // the stream's device must be current
    }
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) return PBCG_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return PBCG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PBCG_OK;
}
}  // namespace

extern "C" {

size_t exdot_noalloc_scratch_bytes(void) { return NOALLOC_BYTES; }

int exdot_noalloc(int64_t n, const double* x, const double* y, double* out, void* stream) {
    if (n < 0 || !out || (n > 0 && (!x || !y))) return PBCG_ERR_INVALID;
    if (n > EXDOT_NOALLOC_MAX_N) return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    void* base = nullptr;
    const int rc = scratch_address(s, &base);
    if (rc != PBCG_OK) return rc;
    const int64_t per = (int64_t)EXDOT_BLOCK * 8;
    const int gmax = n > (int64_t(1) << 25) ? 256 : NOALLOC_GRID;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, gmax));
    // every launched block writes its whole record before the finalize reads it, so
    // nothing in the scratch array has to start at zero
    xd::Site site;
    site.hdr = (xd::RecHdr*)base;
    site.dig = (long long*)((char*)base + NOALLOC_HDR);
    exdot_launch(n, x, y, out, site, s, g, EXDOT_BLOCK, KEXP);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int exdot(int64_t n, const double* x, const double* y, double* out, void* ws, size_t ws_bytes, void* stream) {
    // a standalone dot streams only two vectors: blocks of 1024 threads, 4 elements per lane
    // and trip, 512 blocks up to 2^25 elements and 256 above (at least 8 elements per lane)
    // keep enough loads in flight; the result bits do not depend on the shape
    const int64_t per = (int64_t)EXDOT_BLOCK * 8;
    const int gmax = n > (int64_t(1) << 25) ? 256 : 512;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, gmax));
    return exdot_config(n, x, y, out, g, EXDOT_BLOCK, KEXP, ws, ws_bytes, stream);
}

size_t plain_dot_workspace_bytes(int64_t n) {
    (void)n;
    return align_up((size_t)DOT_GRID_MAX * 4 * sizeof(double), 256) + 256;
}

int plain_dot(int64_t n, const void* x, const void* y, int32_t dtype, void* out, void* ws, size_t ws_bytes,
              void* stream) {
    if (n < 0 || !out || (n > 0 && (!x || !y))) return PBCG_ERR_INVALID;
    if (dtype != PBCG_F64 && dtype != PBCG_F32) return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < plain_dot_workspace_bytes(n) || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    if (dtype == PBCG_F64) {
        TSite<double> site{c.take<double>((size_t)DOT_GRID_MAX * 4)};
        DotsOp<1, FinStore> op{};
        op.a[0] = (const double*)x; op.b[0] = (const double*)y;
        op.fin = FinStore{(double*)out, 1};
        launch_ew_fdot<1>(ElemOf<DotsOp<1, FinStore>>{op}, n, site, nullptr, s);
    } else {
        FSite site{c.take<float>((size_t)DOT_GRID_MAX * 4)};
        FDotsOp<1, FinStoreF> op{};
        op.a[0] = (const float*)x; op.b[0] = (const float*)y;
        op.fin = FinStoreF{(float*)out};
        launch_ew_fdot<1>(op, n, site, nullptr, s);
    }
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

size_t pbcg_phase_workspace_bytes(int32_t n) {
    (void)n;
    return site_bytes(DOT_GRID_MAX);
}

static bool vecs_ok(const pbcg_vectors* V, bool a) {
    if (!V) return false;
    if (a) return V->r && V->w && V->t && V->v && V->rhat && V->p && V->s && V->z && V->q && V->y;
    return V->x && V->p && V->q && V->y && V->t && V->v && V->rhat && V->r && V->w;
}

int pbcg_phase_a(int32_t n, const pbcg_vectors* V, const double* scal, int32_t first, double* dots_out,
                 void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || !scal || !dots_out || (n > 0 && !vecs_ok(V, true))) return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < pbcg_phase_workspace_bytes(n) || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    xd::Site site = carve_site(c, DOT_GRID_MAX);
    PhaseA<FinStore> op{V->r, V->w, V->t, V->v, V->rhat, V->p, V->s, V->z, V->q, V->y, scal, first ? 1 : 0,
                        FinStore{dots_out, 4}};
    launch_ew_dot<4>(op, n, site, nullptr, s);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int pbcg_phase_b(int32_t n, const pbcg_vectors* V, const double* scal, double* dots_out, void* ws,
                 size_t ws_bytes, void* stream) {
    if (n < 0 || !scal || !dots_out || (n > 0 && !vecs_ok(V, false))) return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < pbcg_phase_workspace_bytes(n) || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    xd::Site site = carve_site(c, DOT_GRID_MAX);
    PhaseB<FinStore> op{V->x, V->p, V->q, V->y, V->t, V->v, V->rhat, V->r, V->w, scal, FinStore{dots_out, 3}};
    launch_ew_dot<3>(op, n, site, nullptr, s);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

}  // extern "C"


// ============================================================================ solver driver
namespace {

struct FnCopyF {
    float* dst; const float* src;
    __device__ void operator()(int64_t i) const { dst[i] = src[i]; }
};

struct Work {
    State* st;
    FState* fst;
    xd::Site site;
    FSite fsite;
    TSite<double> dsite;   // partials of the ordinary (plain) FP64 dots
    double *rhat, *r, *w, *t, *p, *s, *z, *q, *y, *v, *tmp, *tmp2, *xbest, *hist;   // xbest: best tested iterate
    float *r32, *rh32, *w32, *t32, *p32, *s32, *z32, *q32, *y32, *v32, *d32, *val32;
    int64_t *a_off, *m_off;   // sliced copies of A and M (null: not reserved)
    int32_t *a_col, *m_col, *a_base, *m_base, *a_perm, *m_perm;
    void *a_val, *m_val;
    size_t need;
    bool ok;
};

bool slicing_on(const pbcg_opts* o) {
    return o && (o->layout == PBCG_LAYOUT_AUTO || o->layout == PBCG_LAYOUT_SORTED || o->layout == PBCG_LAYOUT_SLICED) &&
           o->spmv_kind == PBCG_SPMV_SEQ;
}

Work carve_work(void* ws, size_t bytes, int32_t n, int64_t nnz, const pbcg_opts* o) {
    Carver c(ws, bytes);
    Work W{};
    W.st = c.take<State>(1);
    W.fst = c.take<FState>(1);
    W.site = carve_site(c, DOT_GRID_MAX);
    W.fsite.part = c.take<float>((size_t)DOT_GRID_MAX * 4);
    W.dsite.part = c.take<double>((size_t)DOT_GRID_MAX * 4);
    const size_t N = (size_t)std::max(n, 1);
    double** v64[] = {&W.rhat, &W.r, &W.w, &W.t, &W.p, &W.s, &W.z, &W.q, &W.y, &W.v, &W.tmp, &W.tmp2, &W.xbest};
    for (double** pp : v64) *pp = c.take<double>(N);
    const bool need_hist = o && o->M && o->fallback;
    W.hist = need_hist ? c.take<double>((size_t)std::max(o->max_iter, 1)) : nullptr;
    if (o && o->prec == PBCG_PREC_FP32_IR) {
        float** v32[] = {&W.r32, &W.rh32, &W.w32, &W.t32, &W.p32, &W.s32,
                         &W.z32, &W.q32, &W.y32, &W.v32, &W.d32};
        for (float** pp : v32) *pp = c.take<float>(N);
    }
    if (o && (o->prec == PBCG_PREC_FP32_IR || o->prec == PBCG_PREC_FP32_MATRIX)) {
        // FP32 values in CSR order, or in the sliced order when A has a sliced copy
        W.val32 = c.take<float>((size_t)std::max<int64_t>(slicing_on(o) ? slice_cap(nnz) : nnz, 1));
    }
    if (slicing_on(o)) {
        W.a_off = c.take<int64_t>(slice_off_len(n));
        W.a_col = c.take<int32_t>((size_t)slice_cap(nnz));
        W.a_val = c.take<double>((size_t)slice_cap(nnz));
        W.a_base = c.take<int32_t>((size_t)(slice_cap(nnz) / 256 + 1));
        W.a_perm = c.take<int32_t>(std::max(N, (size_t)nslices(n) * OFS_MAX));   // or the offsets
        if (o->M) {
            W.m_off = c.take<int64_t>(slice_off_len(n));
            W.m_col = c.take<int32_t>((size_t)slice_cap(o->M->nnz));
            W.m_val = c.take<double>((size_t)slice_cap(o->M->nnz));
            W.m_base = c.take<int32_t>((size_t)(slice_cap(o->M->nnz) / 256 + 1));
            W.m_perm = c.take<int32_t>(std::max(N, (size_t)nslices(n) * OFS_MAX));
        }
    }
    W.need = c.off + 256;
    W.ok = c.ok && W.need <= bytes;
    return W;
}

// Bytes an iteration keeps re-reading: the matrices (each SpMV reads them whole) and the
// Krylov vectors.  Above the 256 MB Infinity Cache the phases stream their outputs past the
// caches (non-temporal stores); below it the whole iteration can stay cache-resident and
// plain stores are faster.
constexpr double INFINITY_CACHE_BYTES = 256.0 * 1024 * 1024;

// bytes one SpMV reads of the matrix: CSR, or a sliced copy of `sliced_entries` entries
// (column entries of 2 bytes with d16; none in the offset form, which reads a mask byte per
// row and its slices' offsets instead of the row pointers)
double matrix_bytes(const pbcg_csr* A, int64_t sliced_entries, int value_bytes, bool d16 = false, bool ofs = false) {
    if (!A) return 0.0;
    const double entries = sliced_entries > 0 ? (double)sliced_entries : (double)A->nnz;
    const double ns = nslices(A->n);
    if (sliced_entries > 0 && ofs) return entries * value_bytes + 256.0 * ns + 8.0 * (ns + 1) + 4.0 * OFS_MAX * ns;
    return entries * (value_bytes + (d16 ? 2 : 4)) + 4.0 * ((double)A->n + 1) +
           (sliced_entries > 0 ? 8.0 * (ns + 1) : 0.0);
}

constexpr int CONTINUE = -100;
constexpr int STALLED = 4;   // internal status of a stalled preconditioned solve

struct Driver {
    Mat A;
    Mat M;                 // right preconditioner or null
    const double* b;
    double* x;             // holds y when M != null
    const pbcg_opts* o;
    Work W;
    hipStream_t s;
    int* halt;
    int* seen;             // &st->halt_seen: checked by the SpMVs of the iteration loop
    int batch;
    int max_iter;          // iteration limit of the current run
    int fell_back = 0;     // a fallback (preconditioned) or an FP64 finish (refinement) ran
    int kind;              // SpMV kernel shape
    pbcg_csr A32c;         // FP32 copy of A (refinement) ...
    Mat A32;               // ... with the FP32 sliced values when A is sliced
    Mat Aop;               // the matrix op() applies: A, or A32 (FP32 matrix values)
    int64_t a_entries = 0; // entries of A's sliced copy
    bool nt64 = false;     // stream the FP64 phase outputs past the caches ...
    bool nt32 = false;     // ... and the FP32 ones (working set above the Infinity Cache)
    bool mnt32 = false;    // the FP32 copy of A streams past the cache (larger than it)
    int rr_period = 0;             // residual replacement period of the current run
    double fail_best = INFINITY;   // best true residual of a failed stopping test
    int fail_stag = 0;             // failed tests in a row without improving on it

    // out = A in, or A (M in); `fin` (a pending dot-site finalize) rides on the first SpMV
    template <class Fin = NoFin>
    void op(const double* in, double* out, Fin fin = Fin{}, const int* skip = nullptr) {
        if (o->exact_rows >= 2) {   // no M (checked): every row of A in exactly rounded
            launch_spmv_exact<false>(A, in, nullptr, EpiStore<double>{out}, skip, s, fin);
            return;
        }
        if (M) {
            launch_spmv64(M, in, EpiStore<double>{W.tmp2}, skip, s, kind, fin);
            launch_spmv64(A, W.tmp2, EpiStore<double>{out}, skip, s, kind);
        } else {
            launch_spmv64(Aop, in, EpiStore<double>{out}, skip, s, kind, fin);
        }
    }

    int sync_state(State* h) {
        HIPCHK(hipMemcpyAsync(h, W.st, sizeof(State), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return 0;
    }

    // true residual of the current iterate (x = M y with a preconditioner) -> st->true_rel
    void true_residual_enqueue(int count = 1) {
        const double* xt = x;
        if (M) {
            launch_spmv64(M, x, EpiStore<double>{W.tmp2}, nullptr, s, kind);
            xt = W.tmp2;
        }
        if (o->exact_rows >= 1) {
            EpiResidXDot<FinTrue> epi{W.tmp, FinTrue{W.st, count}};
            launch_spmv_exact_dot<1, true>(A, xt, b, epi, W.site, nullptr, s);
            return;
        }
        EpiResidDot<FinTrue> epi{b, W.tmp, FinTrue{W.st, count}};
        launch_spmv_dot<1>(A, xt, epi, W.site, nullptr, s, kind);
    }

    void dot_enqueue(const double* a, const double* bb, int64_t n) {
        DotsOp<1, FinLastDot> op{};
        op.a[0] = a; op.b[0] = bb; op.fin = FinLastDot{W.st};
        launch_ew_dot<1>(op, n, W.site, nullptr, s);
    }

    // a halted state after init or an iteration: a final status, or CONTINUE
    int handle_halt(State& h) {
        const int n = A->n;
        const int reason = h.reason;
        if (reason & R_CHECK) {
            true_residual_enqueue();
            if (sync_state(&h)) return PBCG_ERR_HIP;
            if (h.true_rel <= h.tol) return PBCG_OK;
            // failed test: the next one 5 iterations on; a new smallest true residual
            // keeps its iterate; 30 failed tests in a row without one: stagnation, and
            // the kept iterate is returned
            launch_single(FnSetCheckIt{W.st, h.iter}, s);
            if (h.true_rel < fail_best) {
                fail_best = h.true_rel;
                fail_stag = 0;
                launch_ew(FnCopy{W.xbest, x}, n, nullptr, s);
            } else if (++fail_stag >= 30) {
                launch_ew(FnCopy{x, W.xbest}, n, nullptr, s);
                return PBCG_STAGNATED;
            }
        }
        if (reason & R_NONFINITE) return PBCG_ERR_NONFINITE;
        if (reason & R_YYZERO) {
            dot_enqueue(W.q, W.q, n);
            if (sync_state(&h)) return PBCG_ERR_HIP;
            if (h.last_dot == 0.0) {  // lucky breakdown: x = x + alpha p completes the iteration
                launch_ew(FnAxpyState{x, W.p, W.st}, n, nullptr, s);
                launch_single(FnIterPlus{W.st}, s);
                true_residual_enqueue();
                if (sync_state(&h)) return PBCG_ERR_HIP;
                return h.true_rel <= h.tol ? PBCG_OK : PBCG_BREAKDOWN;
            }
            return PBCG_BREAKDOWN;
        }
        if (reason & R_BREAKDOWN) return PBCG_BREAKDOWN;
        if (reason & R_STALL) return STALLED;
        if (reason & R_MAXIT) return PBCG_NOT_CONVERGED;
        return CONTINUE;
    }

    void enqueue_iteration_p(bool first, long long it) {
        if (nt64) enqueue_iteration_p_t<true>(first, it);
        else enqueue_iteration_p_t<false>(first, it);
    }

    template <bool NT>
    void enqueue_iteration_p_t(bool first, long long it) {
        const int n = A->n;
        const double* scal = &W.st->alpha;
        PhaseA<FinOmega, NT> pa{W.r, W.w, W.t, W.v, W.rhat, W.p, W.s, W.z, W.q, W.y, scal, first ? 1 : 0,
                                FinOmega{W.st, 1}};
        PhaseB<FinPhaseB, NT> pb{x, W.p, W.q, W.y, W.t, W.v, W.rhat, W.r, W.w, scal, FinPhaseB{W.st}};
        if (o->dots == PBCG_DOTS_PLAIN) {
            auto fa = launch_ew_fdot_deferred<4>(ElemOf<PhaseA<FinOmega, NT>>{pa}, n, W.dsite, halt, s, seen);
            op(W.z, W.v, fa, seen);
            auto fb = launch_ew_fdot_deferred<3>(ElemOf<PhaseB<FinPhaseB, NT>>{pb}, n, W.dsite, halt, s, seen);
            op(W.w, W.t, fb, seen);
            return;
        }
        hipEvent_t* ev = kernel_events(it);
        if (ev) { g_kev[0] = ev[0]; g_kev[1] = ev[1]; }
        auto fa = launch_ew_dot_deferred<4, DOT_GRID_DEFAULT>(pa, n, W.site, halt, s, 0, DOT_BLOCK, KEXP, seen);
        if (ev) { g_kev[0] = ev[2]; g_kev[1] = ev[3]; }
        op(W.z, W.v, fa, seen);           // v = A z; omega is finalized by its block 0
        if (ev) { g_kev[0] = ev[4]; g_kev[1] = ev[5]; }
        auto fb = launch_ew_dot_deferred<3, DOT_GRID_DEFAULT>(pb, n, W.site, halt, s, 0, DOT_BLOCK, KEXP, seen);
        if (ev) { g_kev[0] = ev[6]; g_kev[1] = ev[7]; }
        op(W.w, W.t, fb, seen);           // t = A w; beta, alpha finalized by its block 0
        g_kev[0] = g_kev[1] = nullptr;
    }

    // The caller's timing events for iteration `it` (0-based; iteration 0 copies instead
    // of updating and is not timed), or null.
    hipEvent_t* kernel_events(long long it) const {
        if (!o->kernel_events || o->kernel_events_len < 8 || M || o->dots != PBCG_DOTS_EXACT ||
            kind != PBCG_SPMV_SEQ)
            return nullptr;
        if (it < 1 || it > o->kernel_events_len / 8) return nullptr;
        return (hipEvent_t*)o->kernel_events + 8 * (it - 1);
    }

    // After completed iteration `it` (skipped if it halted): the periodic true residual
    // for the history, then the residual replacement.
    void enqueue_after_iteration(long long it) {
        if (o->true_every > 0 && o->true_history && it % o->true_every == 0) {
            const long long k = it / o->true_every - 1;
            if (k < o->true_history_len) {
                if (o->exact_rows >= 1) {
                    EpiResidXDot<FinTrueHist> epi{W.tmp, FinTrueHist{W.st, o->true_history + k}};
                    launch_spmv_exact_dot<1, true>(A, x, b, epi, W.site, halt, s);
                } else {
                    EpiResidDot<FinTrueHist> epi{b, W.tmp, FinTrueHist{W.st, o->true_history + k}};
                    launch_spmv_dot<1>(A, x, epi, W.site, halt, s, kind);
                }
            }
        }
        if (rr_period > 0 && it % rr_period == 0) enqueue_replacement();
    }

    // Residual replacement after a completed iteration (skipped if the iteration halted):
    // r = b - A x, w = A r, t = A w, s = A p, z = A s, v = A z; scalars unchanged.
    void enqueue_replacement() {
        if (o->exact_rows >= 1)
            launch_spmv_exact<true>(A, x, b, EpiResidX<double>{W.r, nullptr, nullptr}, halt, s);
        else
            launch_spmv64(A, x, EpiResid<double>{b, W.r, nullptr, nullptr}, halt, s, kind);
        op(W.r, W.w, NoFin{}, halt);
        op(W.w, W.t, NoFin{}, halt);
        op(W.p, W.s, NoFin{}, halt);
        op(W.s, W.z, NoFin{}, halt);
        op(W.z, W.v, NoFin{}, halt);
    }

    void enqueue_iteration_b() {
        if (nt64) enqueue_iteration_b_t<true>();
        else enqueue_iteration_b_t<false>();
    }

    template <bool NT>
    void enqueue_iteration_b_t() {
        const int n = A->n;
        const double* scal = &W.st->alpha;
        launch_ew(FnPUpdate<NT>{W.p, W.r, W.s, W.st}, n, halt, s);
        launch_spmv_dot<1>(A, W.p, EpiSDot<NT>{W.s, W.rhat, FinAlphaB{W.st}}, W.site, halt, s, kind);
        launch_ew(FnQ<NT>{W.q, W.r, W.s, scal}, n, halt, s);
        launch_spmv_dot<2>(A, W.q, EpiYDot<NT>{W.y, W.q, FinOmega{W.st, 0}}, W.site, halt, s, kind);
        OpBiCGStabXR<NT> ox{x, W.p, W.q, W.y, W.rhat, W.r, scal, FinBiCGStabXR{W.st}};
        launch_ew_dot<2>(ox, n, W.site, halt, s);
    }

    // FP64 p-BiCGStab / BiCGStab on A (or A.M).  x: x0 in, iterate out (y with M).
    int run_fp64(State& h) {
        const int n = A->n;
        fail_best = INFINITY;
        fail_stag = 0;
        const bool bicg = o->alg == PBCG_ALG_BICGSTAB;
        double* hist = o->history;
        const int hist_len = hist ? o->history_len : 0;
        const bool stall_on = M && o->fallback && W.hist;
        const int window = o->stall_window > 0 ? o->stall_window : 200;
        launch_single(FnInitState{W.st, o->tol, max_iter, hist, hist_len, stall_on ? window : 0,
                                  stall_on ? W.hist : nullptr}, s);
        {
            DotsOp<1, FinNormB> nb{};
            nb.a[0] = b; nb.b[0] = b; nb.fin = FinNormB{W.st};
            launch_ew_dot<1>(nb, n, W.site, nullptr, s);
        }
        if (M) {  // y0 = 0, r0 = b
            launch_ew(FnZero{x}, n, nullptr, s);
            launch_ew(FnCopy3{W.r, W.rhat, bicg ? W.p : nullptr, b}, n, nullptr, s);
        } else if (o->exact_rows >= 1) {
            launch_spmv_exact<true>(A, x, b, EpiResidX<double>{W.r, W.rhat, bicg ? W.p : nullptr}, nullptr, s);
        } else {
            launch_spmv64(A, x, EpiResid<double>{b, W.r, W.rhat, bicg ? W.p : nullptr}, nullptr, s, kind);
        }
        if (!bicg) {
            op(W.r, W.w, NoFin{}, halt);
            op(W.w, W.t, NoFin{}, halt);
            DotsOp<3, FinInitP> d3{};
            d3.a[0] = W.rhat; d3.b[0] = W.r;
            d3.a[1] = W.rhat; d3.b[1] = W.w;
            d3.a[2] = W.r;    d3.b[2] = W.r;
            d3.fin = FinInitP{W.st};
            if (o->dots == PBCG_DOTS_PLAIN) launch_ew_fdot<3>(ElemOf<DotsOp<3, FinInitP>>{d3}, n, W.dsite, halt, s);
            else launch_ew_dot<3>(d3, n, W.site, halt, s);
        } else {
            DotsOp<2, FinInitB> d2{};
            d2.a[0] = W.rhat; d2.b[0] = W.r;
            d2.a[1] = W.r;    d2.b[1] = W.r;
            d2.fin = FinInitB{W.st};
            launch_ew_dot<2>(d2, n, W.site, halt, s);
        }
        HIPCHK(hipGetLastError());
        if (sync_state(&h)) return PBCG_ERR_HIP;
        if (h.halt) {
            if (h.reason & R_ZERO_RHS) {
                launch_ew(FnZero{x}, n, nullptr, s);
                return PBCG_OK;
            }
            int r = handle_halt(h);
            if (r != CONTINUE) return r;
            launch_single(FnResume{W.st}, s);
        }
        if (max_iter == 0) return PBCG_NOT_CONVERGED;
        bool first = true;
        long long it_enq = 0;   // iterations enqueued since the start (replacement schedule)
        int polled = 0, batches = 0;
        // device-side halts end the loop; this bound only guards against a broken state
        const long long limit = (long long)max_iter + 4LL * batch + 64;
        long long enqueued = 0;
        int nb = batch;         // after a failed true-residual test the solve halts every 5
                                // iterations: batches of 5 keep the no-op launches queued
                                // behind each halt to one batch
        while (true) {
            if (enqueued > limit) return PBCG_ERR_HIP;
            enqueued += nb;
            for (int k = 0; k < nb; ++k) {
                if (bicg) enqueue_iteration_b();
                else enqueue_iteration_p(first, it_enq);
                first = false;
                ++it_enq;
                if (!bicg) enqueue_after_iteration(it_enq);
            }
            HIPCHK(hipGetLastError());
            const int slot = batches & 1;
            HIPCHK(hipMemcpyAsync(&g_pin.s[slot], W.st, sizeof(State), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(g_pin.ev[slot], s));
            ++batches;
            if (batches - polled >= 2) {  // keep one batch queued behind the one being waited on
                const int ps = polled & 1;
                HIPCHK(hipEventSynchronize(g_pin.ev[ps]));
                ++polled;
                if (g_pin.s[ps].halt) {
                    if (sync_state(&h)) return PBCG_ERR_HIP;   // later batches were no-ops
                    int r = handle_halt(h);
                    if (r != CONTINUE) return r;
                    if (h.reason & R_CHECK) nb = std::min(batch, 5);
                    launch_single(FnResume{W.st}, s);
                    polled = batches;
                    enqueued = h.iter;  // batches queued behind the halt were no-ops
                    it_enq = h.iter;
                    // the work after the halted iteration was skipped with it
                    if (!bicg && h.iter > 0) enqueue_after_iteration(h.iter);
                }
            }
        }
    }

    // One FP32 iteration: phase A, v = A z, phase B, t = A w.
    template <bool NT>
    void enqueue_iteration_f32(bool first) {
        const int n = A->n;
        FState* fs = W.fst;
        const float* scal = &fs->alpha;
        FPhaseA<FFinOmega, NT> pa{W.r32, W.w32, W.t32, W.v32, W.rh32, W.p32, W.s32, W.z32, W.q32, W.y32,
                                  scal, first ? 1 : 0, FFinOmega{fs}};
        auto fa = launch_ew_fdot_deferred<4>(pa, n, W.fsite, &fs->halt, s, &fs->halt_seen);
        launch_spmv32c(A32, W.z32, EpiStore<float>{W.v32}, &fs->halt_seen, s, fa);
        FPhaseB<FFinRU, NT> pb{W.d32, W.p32, W.q32, W.y32, W.t32, W.v32, W.rh32, W.r32, W.w32, scal,
                               FFinRU{fs}};
        auto fb = launch_ew_fdot_deferred<3>(pb, n, W.fsite, &fs->halt, s, &fs->halt_seen);
        launch_spmv32c(A32, W.w32, EpiStore<float>{W.t32}, &fs->halt_seen, s, fb);
    }

    // FP32 p-BiCGStab (Algorithm 2) on A32 with right-hand side W.r32, x0 = 0 -> W.d32.
    // FP32 iterations (phase A, v = A z, phase B, t = A w) until a finalizer sets a stop
    // reason; returns the final FState in hf.
    int run_fp32(FState& hf, bool first) {
        FState* fs = W.fst;
        int polled = 0, batches = 0;
        // short batches: every reliable update halts the FP32 run, and the iterations
        // queued behind a halt (up to two batches) run as no-op launches
        const int nb = std::min(batch, IR_BATCH);
        const long long limit = (long long)std::max(o->max_iter, 1) + 4LL * nb + 64;
        long long enqueued = 0;
        while (true) {
            if (enqueued > limit) return PBCG_ERR_HIP;   // a stop reason must have come (MAXIT)
            enqueued += nb;
            for (int k = 0; k < nb; ++k) {
                if (nt32) enqueue_iteration_f32<true>(first);
                else enqueue_iteration_f32<false>(first);
                first = false;
            }
            HIPCHK(hipGetLastError());
            const int slot = batches & 1;
            HIPCHK(hipMemcpyAsync(&g_pin.f[slot], fs, sizeof(FState), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(g_pin.ev[slot], s));
            ++batches;
            if (batches - polled >= 2) {
                const int ps = polled & 1;
                HIPCHK(hipEventSynchronize(g_pin.ev[ps]));
                ++polled;
                if (g_pin.f[ps].halt) {
                    HIPCHK(hipMemcpyAsync(&hf, fs, sizeof(FState), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                    return 0;
                }
            }
        }
    }

    // r = b - A x (row-sequential FP64 SpMV) and nu = sqrt(exdot(r, r)) -> st, h
    int true_residual_ir(State& h) {
        EpiResidDot<FinIR> epi{b, W.r, FinIR{W.st}};
        launch_spmv_dot<1>(A, x, epi, W.site, nullptr, s, kind);
        return sync_state(&h);
    }

    // FP64 iterative refinement around FP32 p-BiCGStab with reliable updates: the FP32
    // Krylov process runs on r / nu and accumulates a correction d; each time it stops
    // (its residual dropped by inner_tol, it looks converged, a breakdown or a stall),
    // x = x + nu d, the true residual is formed in FP64 with an exact norm, and the FP32
    // state is rebuilt from it -- continued (p rescaled; w, t, s, z, v recomputed) or,
    // after a breakdown or stall, restarted.  An update that does not improve on the
    // best iterate means FP32 has reached its accuracy floor (about u32 cond(A)): the
    // solve then finishes in FP64 p-BiCGStab from the best iterate.
    // A32: A with its values rounded to FP32 (in the sliced order when A is sliced)
    void make_a32() {
        A32c = *A.csr;
        A32c.val = W.val32;
        A32c.val_type = PBCG_F32;
        if (A.sl.off) {   // the FP32 values in the sliced order (padding casts to 0)
            launch_ew(FnCastVal{W.val32, (const double*)A.sl.val}, a_entries, nullptr, s);
            SliceView v32 = A.sl;
            v32.val = W.val32;
            v32.nt = mnt32;
            A32 = Mat(&A32c, v32);
        } else {
            launch_ew(FnCastVal{W.val32, (const double*)A->val}, A->nnz, nullptr, s);
            A32 = Mat(&A32c);
        }
    }

    int run_ir(State& h, int& outer, int& inner_total) {
        const int n = A->n;
        FState* fs = W.fst;
        launch_single(FnInitState{W.st, o->tol, o->max_iter, nullptr, 0, 0, nullptr}, s);
        make_a32();
        {
            DotsOp<1, FinNormB> nb{};
            nb.a[0] = b; nb.b[0] = b; nb.fin = FinNormB{W.st};
            launch_ew_dot<1>(nb, n, W.site, nullptr, s);
        }
        HIPCHK(hipGetLastError());
        if (sync_state(&h)) return PBCG_ERR_HIP;
        outer = 0;
        inner_total = 0;
        if (h.reason & R_ZERO_RHS) {
            launch_ew(FnZero{x}, n, nullptr, s);
            return PBCG_OK;
        }
        if (h.reason & R_NONFINITE) return PBCG_ERR_NONFINITE;
        const double normb = h.normb;
        const int max_outer = o->max_outer > 0 ? o->max_outer : IR_MAX_UPDATES;
        const float delta = (float)(o->inner_tol > 0.0 ? o->inner_tol : IR_DELTA);
        double* x_best = W.p;   // the FP64 p vector is free during the refinement
        if (true_residual_ir(h)) return PBCG_ERR_HIP;
        double nu = h.last_dot;
        if (!std::isfinite(nu)) return PBCG_ERR_NONFINITE;
        if (h.true_rel <= o->tol) return PBCG_OK;
        launch_ew(FnCopy{x_best, x}, n, nullptr, s);
        double nu_best = nu;
        int bad = 0;
        bool restart = true;
        float sigma = 1.0f;
        launch_single(FnInitFState{fs, delta, std::max(o->max_iter, 1), IR_INNER_STALL}, s);
        auto finish = [&]() -> int {   // FP64 p-BiCGStab from the best iterate
            launch_ew(FnCopy{x, x_best}, n, nullptr, s);
            fell_back = 1;
            max_iter = IR_FP64_FINISH;
            rr_period = IR_FINISH_RR;   // the restart point's gap must not limit the finish
            const int st = run_fp64(h);
            inner_total += h.iter;
            return st;
        };
        while (true) {
            // rebuild the FP32 state from r / nu
            const float lim = (float)(o->tol * normb / nu);
            launch_ew(FnCastScaled{W.r32, W.r, W.st}, n, nullptr, s);
            launch_spmv32c(A32, W.r32, EpiStore<float>{W.w32}, nullptr, s);
            launch_spmv32c(A32, W.w32, EpiStore<float>{W.t32}, nullptr, s);
            launch_single(FnSetFState{fs, lim}, s);
            FState hf{};
            if (!restart) {
                launch_ew(FnScaleF{W.p32, sigma}, n, nullptr, s);
                launch_spmv32c(A32, W.p32, EpiStore<float>{W.s32}, nullptr, s);
                launch_spmv32c(A32, W.s32, EpiStore<float>{W.z32}, nullptr, s);
                launch_spmv32c(A32, W.z32, EpiStore<float>{W.v32}, nullptr, s);
                FDotsOp<4, FFinReplace> d{};
                d.a[0] = W.rh32; d.b[0] = W.r32;
                d.a[1] = W.rh32; d.b[1] = W.w32;
                d.a[2] = W.rh32; d.b[2] = W.s32;
                d.a[3] = W.rh32; d.b[3] = W.z32;
                d.fin = FFinReplace{fs};
                launch_ew_fdot<4>(d, n, W.fsite, nullptr, s);
                HIPCHK(hipMemcpyAsync(&hf, fs, sizeof(FState), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                if (hf.halt) {              // no usable alpha: restart from the same residual
                    restart = true;
                    launch_single(FnSetFState{fs, lim}, s);
                }
            }
            if (restart) {
                launch_ew(FnCopyF{W.rh32, W.r32}, n, nullptr, s);
                FDotsOp<2, FFinRestart> d{};
                d.a[0] = W.rh32; d.b[0] = W.r32;
                d.a[1] = W.rh32; d.b[1] = W.w32;
                d.fin = FFinRestart{fs};
                launch_ew_fdot<2>(d, n, W.fsite, nullptr, s);
                HIPCHK(hipMemcpyAsync(&hf, fs, sizeof(FState), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                if (hf.halt) return finish();
            }
            launch_ew(FnZeroF{W.d32}, n, nullptr, s);
            if (run_fp32(hf, restart)) return PBCG_ERR_HIP;
            const int reason = hf.reason;
            if (reason & R_YYZERO) {        // (y, y) = 0: d = d + alpha p completes the iteration
                launch_ew(FnFAxpyState{W.d32, W.p32, fs}, n, nullptr, s);
                launch_single(FnFIterPlus{fs}, s);
            }
            inner_total = hf.iter + ((reason & R_YYZERO) ? 1 : 0);
            // reliable update
            launch_ew(FnIRUpdate{x, W.d32, W.st}, n, nullptr, s);
            if (true_residual_ir(h)) return PBCG_ERR_HIP;
            ++outer;
            double nu_new = h.last_dot;
            if (o->trace)
                std::fprintf(stderr, "pbicgstab ir: update %d after %d FP32 iterations: reason 0x%x rec %.3e "
                             "true/previous %.3e true/||b|| %.3e%s\n", outer, inner_total, reason, (double)hf.rec,
                             nu_new / nu, h.true_rel, restart ? " (restarted)" : "");
            if (!std::isfinite(nu_new)) return finish();
            if (h.true_rel <= o->tol) return PBCG_OK;
            restart = (reason & (R_BREAKDOWN | R_NONFINITE | R_STALL | R_YYZERO)) != 0;
            if (nu_new < nu_best) {
                nu_best = nu_new;
                bad = 0;
                launch_ew(FnCopy{x_best, x}, n, nullptr, s);
            } else {
                ++bad;
                restart = true;
                launch_ew(FnCopy{x, x_best}, n, nullptr, s);
                if (true_residual_ir(h)) return PBCG_ERR_HIP;
                nu_new = h.last_dot;
            }
            if (bad >= IR_MAX_BAD || outer >= max_outer || (reason & R_MAXIT)) return finish();
            sigma = (float)(nu / nu_new);
            nu = nu_new;
        }
    }
};

}  // namespace

extern "C" {

size_t pbicgstab_workspace_bytes(int32_t n, int64_t nnz, const pbcg_opts* opts) {
    pbcg_opts d;
    if (!opts) { pbcg_default_opts(&d); opts = &d; }
    Work W = carve_work(nullptr, SIZE_MAX, n, nnz, opts);
    return W.need;
}

int pbicgstab_solve(const pbcg_csr* A, const double* b, double* x, const pbcg_opts* opts, pbcg_info* info,
                    void* ws, size_t ws_bytes, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (info) std::memset(info, 0, sizeof(*info));
    if (!csr_ok(A) || !opts) return PBCG_ERR_INVALID;
    if (A->n > 0 && (!b || !x)) return PBCG_ERR_INVALID;
    if (opts->max_iter < 0 || !(opts->tol >= 0.0)) return PBCG_ERR_INVALID;
    if (opts->kernel_events_len < 0 || opts->kernel_events_len % 8 != 0 ||
        (opts->kernel_events_len > 0 && !opts->kernel_events))
        return PBCG_ERR_INVALID;
    if (opts->alg != PBCG_ALG_PBICGSTAB && opts->alg != PBCG_ALG_BICGSTAB) return PBCG_ERR_INVALID;
    if (opts->prec != PBCG_PREC_FP64 && opts->prec != PBCG_PREC_FP32_IR && opts->prec != PBCG_PREC_FP32_MATRIX)
        return PBCG_ERR_INVALID;
    if (opts->prec == PBCG_PREC_FP32_MATRIX &&
        (opts->M || opts->alg != PBCG_ALG_PBICGSTAB || A->val_type != PBCG_F64 || opts->exact_rows != 0))
        return PBCG_ERR_INVALID;
    if (opts->M && (!csr_ok(opts->M) || opts->M->n != A->n)) return PBCG_ERR_INVALID;
    if (opts->M && opts->alg != PBCG_ALG_PBICGSTAB) return PBCG_ERR_INVALID;
    if (opts->prec == PBCG_PREC_FP32_IR && (opts->M || opts->alg != PBCG_ALG_PBICGSTAB || A->val_type != PBCG_F64))
        return PBCG_ERR_INVALID;
    if (opts->history && opts->history_len < 0) return PBCG_ERR_INVALID;
    if (opts->spmv_kind < PBCG_SPMV_SEQ || opts->spmv_kind > PBCG_SPMV_WAVE) return PBCG_ERR_INVALID;
    if (opts->dots != PBCG_DOTS_EXACT && opts->dots != PBCG_DOTS_PLAIN) return PBCG_ERR_INVALID;
    if (opts->rr_period < 0) return PBCG_ERR_INVALID;
    if (opts->layout < PBCG_LAYOUT_AUTO || opts->layout > PBCG_LAYOUT_SLICED) return PBCG_ERR_INVALID;
    if (opts->exact_rows < 0 || opts->exact_rows > 2) return PBCG_ERR_INVALID;
    if (opts->exact_rows > 0 && (opts->M || opts->alg != PBCG_ALG_PBICGSTAB || opts->prec != PBCG_PREC_FP64))
        return PBCG_ERR_INVALID;
    if (opts->true_every < 0 || (opts->true_history && opts->true_history_len < 0)) return PBCG_ERR_INVALID;
    if (opts->true_every > 0 && opts->true_history &&
        (opts->M || opts->alg != PBCG_ALG_PBICGSTAB || opts->prec != PBCG_PREC_FP64))
        return PBCG_ERR_INVALID;
    if ((opts->dots == PBCG_DOTS_PLAIN || opts->rr_period > 0) &&
        (opts->M || opts->alg != PBCG_ALG_PBICGSTAB ||
         (opts->prec != PBCG_PREC_FP64 && opts->prec != PBCG_PREC_FP32_MATRIX)))
        return PBCG_ERR_INVALID;
    if (!ws || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    Work W = carve_work(ws, ws_bytes, A->n, A->nnz, opts);
    if (!W.ok) return PBCG_ERR_WORKSPACE;
    if (A->n == 0) {
        if (info) info->status = PBCG_OK;
        return PBCG_OK;
    }
    if (pin_init()) return PBCG_ERR_HIP;
    Driver D{};
    D.A = A; D.M = opts->M; D.b = b; D.x = x; D.o = opts; D.W = W; D.s = (hipStream_t)stream;
    D.halt = &W.st->halt;
    D.seen = &W.st->halt_seen;
    D.batch = opts->batch > 0 ? opts->batch : 16;
    D.kind = opts->spmv_kind;
    D.max_iter = opts->max_iter;
    D.rr_period = opts->rr_period;
    int sliced = 0;   // bit 0: A, bit 1: M use a sliced copy
    int64_t m_entries = 0;
    if (slicing_on(opts)) {
        bool a16 = false, m16 = false;
        // AUTO: the 256-row sliced copy when its padding is small (stencils), else CSR.
        // SORTED: the row-sorted copy (64-row slices of rows ordered by length within
        // windows of 4096 rows) when its padding fits.  (Measured on the random 10^6
        // matrix: 157 us per SpMV on the row-sorted copy against 112 us for the staged CSR
        // kernel, so AUTO does not choose it.)
        auto make = [&](const pbcg_csr* B, int64_t* off, int32_t* col, void* val, int32_t* base, int32_t* perm,
                        bool* d16, SliceView* v, int64_t* entries, int* sorted) -> int {
            const int64_t cap = slice_cap(B->nnz);
            int64_t t = cap + 1;
            // AUTO: the offset form first (banded / stencil rows); its mask bytes live in the
            // column array, its offsets in the permutation array
            if (opts->layout == PBCG_LAYOUT_AUTO && (int64_t)nslices(B->n) * 256 <= 4 * cap) {
                t = build_ofs(B, off, perm, (uint8_t*)col, val, cap, D.s);
                if (t < 0) return -1;
                if (t > 0 && t <= cap) {
                    *v = SliceView{off, nullptr, val};
                    v->mask = (const uint8_t*)col;
                    v->ofs = perm;
                    *entries = t;
                    *d16 = false;
                    *sorted = 2;
                    return 1;
                }
            }
            if (opts->layout != PBCG_LAYOUT_SORTED) {
                t = build_slices(B, off, col, val, base, cap, D.s, true, d16);
                if (t < 0) return -1;
                if (t <= cap) {
                    *v = SliceView{off, col, val};
                    v->d16 = *d16;
                    v->base = base;
                    *entries = t;
                    return 1;
                }
            }
            *d16 = false;
            if (opts->layout != PBCG_LAYOUT_SORTED) return 0;
            t = build_wslices(B, perm, off, col, val, cap, D.s);
            if (t < 0) return -1;
            if (t > cap) return 0;
            *v = SliceView{off, col, val};
            v->perm = perm;
            *entries = t;
            *sorted = 1;
            return 1;
        };
        int a_sorted = 0, m_sorted = 0;
        const int ra = make(A, W.a_off, W.a_col, W.a_val, W.a_base, W.a_perm, &a16, &D.A.sl, &D.a_entries, &a_sorted);
        if (ra < 0) return PBCG_ERR_HIP;
        if (ra > 0) sliced |= 1 | (a_sorted == 1 ? 16 : 0) | (a_sorted == 2 ? 64 : 0);
        if (opts->M) {
            const int rm = make(opts->M, W.m_off, W.m_col, W.m_val, W.m_base, W.m_perm, &m16, &D.M.sl, &m_entries,
                                &m_sorted);
            if (rm < 0) return PBCG_ERR_HIP;
            if (rm > 0) sliced |= 2 | (m_sorted == 1 ? 32 : 0) | (m_sorted == 2 ? 128 : 0);
        }
    }
    {
        const int64_t ma = (sliced & 1) ? D.a_entries : 0;
        const int vb = (A->val_type == PBCG_F64 && opts->prec != PBCG_PREC_FP32_MATRIX) ? 8 : 4;
        const bool a16 = D.A.sl.d16, m16 = D.M.sl.d16;
        const bool ao = D.A.sl.mask != nullptr, mo = D.M.sl.mask != nullptr;
        double ws64 = matrix_bytes(A, ma, vb, a16, ao) + 12.0 * 8.0 * A->n;
        if (opts->M) {
            const int64_t mm = (sliced & 2) ? m_entries : 0;
            ws64 += matrix_bytes(opts->M, mm, opts->M->val_type == PBCG_F64 ? 8 : 4, m16, mo) + 8.0 * A->n;
        }
        D.nt64 = ws64 > INFINITY_CACHE_BYTES;
        D.nt32 = matrix_bytes(A, ma, 4, a16, ao) + 11.0 * 4.0 * A->n > INFINITY_CACHE_BYTES;
        // a matrix that does not fit the cache at all streams past it as well (measured on
        // 256^3: 1.79 -> 1.69 s; a matrix that fits stays resident instead)
        D.A.sl.nt = (sliced & 1) && matrix_bytes(A, ma, vb, a16, ao) > INFINITY_CACHE_BYTES;
        D.mnt32 = (sliced & 1) && matrix_bytes(A, ma, 4, a16, ao) > INFINITY_CACHE_BYTES;
        if (opts->M && (sliced & 2))
            D.M.sl.nt = matrix_bytes(opts->M, m_entries, opts->M->val_type == PBCG_F64 ? 8 : 4, m16, mo) >
                        INFINITY_CACHE_BYTES;
        if (a16) sliced |= 4;
        if (m16) sliced |= 8;
    }
    D.Aop = D.A;
    if (opts->prec == PBCG_PREC_FP32_MATRIX) {
        // the iterations apply A's values rounded to FP32 (4 bytes per entry instead of 8);
        // the residual replacement against the FP64 A keeps the iterate on A x = b
        D.make_a32();
        D.Aop = D.A32;
        if (D.rr_period <= 0) D.rr_period = FP32M_RR;
    }
    State h{};
    int status;
    int outer = 0, inner_total = 0;
    int fell_back = 0, iters_before = 0;
    if (opts->prec == PBCG_PREC_FP32_IR) {
        status = D.run_ir(h, outer, inner_total);
        fell_back = D.fell_back;
    } else {
        status = D.run_fp64(h);
        if (D.M && opts->fallback &&
            (status == PBCG_BREAKDOWN || status == PBCG_ERR_NONFINITE || status == STALLED)) {
            // the true residual judges between x0 = 0 and x = M y; restart unpreconditioned
            D.true_residual_enqueue();          // x = M y lands in tmp2
            if (D.sync_state(&h)) return PBCG_ERR_HIP;
            if (std::isfinite(h.true_rel) && h.true_rel < 1.0) launch_ew(FnCopy{x, W.tmp2}, A->n, nullptr, D.s);
            else launch_ew(FnZero{x}, A->n, nullptr, D.s);
            iters_before = h.iter;
            D.M = nullptr;
            D.max_iter = std::max(opts->max_iter - iters_before, 0);
            fell_back = 1;
            status = D.run_fp64(h);
        }
    }
    if (status == STALLED) status = PBCG_BREAKDOWN;  // only reachable without a fallback
    if (status != PBCG_ERR_HIP) {
        const bool have_true = (opts->prec == PBCG_PREC_FP32_IR && !fell_back) ||
                               (status == PBCG_OK && (h.reason & (R_CHECK | R_YYZERO)));
        if (!have_true && !(h.reason & R_ZERO_RHS)) {
            D.true_residual_enqueue(0);   // the reported value, not a stopping test
        }
        if (D.M) {  // x = M y
            launch_spmv64(D.M, x, EpiStore<double>{W.tmp2}, nullptr, D.s, D.kind);
            launch_ew(FnCopy{x, W.tmp2}, A->n, nullptr, D.s);
        }
        if (opts->r_out)
            (void)hipMemcpyAsync(opts->r_out, W.r, sizeof(double) * (size_t)A->n, hipMemcpyDeviceToDevice, D.s);
        if (D.sync_state(&h)) status = PBCG_ERR_HIP;
        if (hipGetLastError() != hipSuccess) status = PBCG_ERR_HIP;
    }
    if (info) {
        const bool zr = (h.reason & R_ZERO_RHS) != 0;
        info->status = status;
        info->iterations = opts->prec == PBCG_PREC_FP32_IR ? inner_total : h.iter + iters_before;
        info->fell_back = fell_back;
        info->sliced = sliced;
        info->sliced_entries = (sliced & 1) ? D.a_entries : 0;
        info->outer_iterations = outer;
        info->true_checks = h.true_checks;
        info->true_relres = zr ? 0.0 : h.true_rel;
        info->rec_relres = zr ? 0.0 : ((opts->prec == PBCG_PREC_FP32_IR && !fell_back) ? h.true_rel : h.rec);
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // extern "C"
