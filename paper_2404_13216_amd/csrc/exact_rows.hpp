// Exactly rounded SpMV rows (gfx950, wave64): every row's sum formed exactly and rounded
// once to nearest even, so y = A x (or r = b - A x) depends on no summation order.
//
//  * exact_row_fast     one lane per row: the row's exact sum in a window of 8 registers
//                       of 32-bit chunks, rounded by the lane itself (rows whose terms
//                       span a few chunks: the common case);
//  * exact_row          16 lanes per row: the row's long accumulator in LDS (any row);
//  * spmv_exact_kernel  short rows (mean length up to 12): blocks of 256 threads over
//                       chunks of 256 rows, the fast path first, then the rows it hands
//                       back in groups of 16 lanes; longer rows: every row in groups of
//                       16 lanes;
//  * spmv_exact_dot_kernel  the same with D exact dots of the rows in the epilogue.
#pragma once
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace pbcg {

// The reproducible-reduction idea of the paper's exact inner products (exact accumulation,
// one rounding; Section 2) applied to the rows of A x.
//
// LDS path: 16 lanes (one DPP row of the wave) take one matrix row: each lane deposits
// its products as exact integers
// (TwoProd is not needed: the 106-bit product goes straight into the row's long
// accumulator of 32-bit chunks in LDS, integer additions commute), the group finds the
// chunk range it touched, and its leader rounds the range once (the exact dot's
// rounding).  RESID: the row value is b_i - (A x)_i as one exact sum (b_i enters as a
// term), rounded once.
constexpr int XR_GROUP = 16;                   // lanes per matrix row
constexpr int XR_ROWS = 256 / XR_GROUP;        // rows in flight per 256-thread block
constexpr int XR_SMEM = XR_ROWS * xd::NCH * 8 + XR_ROWS * 4;

__device__ __forceinline__ int xr_row_max(int v) { return -xd::row_min_i(-v); }

__device__ __forceinline__ void xr_flag_nonfinite(uint32_t* flag, double a, double x) {
    uint32_t f;
    if (isnan(a) || isnan(x) || a == 0.0 || x == 0.0) f = xd::F_NAN;
    else f = ((a > 0.0) == (x > 0.0)) ? xd::F_PINF : xd::F_NINF;
    atomicOr(flag, f);
}

// One row per 16-lane group (row < 0: the group idles).  acc: the group's NCH chunks, zero
// on entry and zero again on return; flag: the group's non-finite flags (likewise).  All
// 64 lanes of the wave call it together; the group leader (gl == 0) gets the value.
template <class VT, bool RESID>
__device__ __forceinline__ double exact_row(int row, const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ ci, const VT* __restrict__ val,
                                            const double* __restrict__ x, const double* __restrict__ b,
                                            unsigned long long* acc, uint32_t* flag, int gl) {
    int lo = INT_MAX, hi = -1;
    if (row >= 0) {
        const int a = rp[row], e = rp[row + 1];
        for (int k = a + gl; k < e; k += XR_GROUP) {
            const double av = (double)val[k], xv = x[ci[k]];
            if (!(isfinite(av) && isfinite(xv))) {
                xr_flag_nonfinite(flag, RESID ? -av : av, xv);
            } else if (av != 0.0 && xv != 0.0) {
                uint64_t m;
                int Pa, Px;
                bool ng;
                xd::decompose(av, m, Pa, ng);
                xd::decompose(xv, m, Px, ng);
                const int c = (Pa + Px - xd::BIAS) >> 5;     // lowest chunk of the product
                lo = min(lo, c);
                hi = max(hi, c + 4);
                xd::deposit_product(acc, RESID ? -av : av, xv);
            }
        }
        if constexpr (RESID) {
            if (gl == 0) {
                const double bv = b[row];
                if (!isfinite(bv)) {
                    xr_flag_nonfinite(flag, bv, 1.0);
                } else if (bv != 0.0) {
                    uint64_t m;
                    int P;
                    bool ng;
                    xd::decompose(bv, m, P, ng);
                    lo = min(lo, P >> 5);
                    hi = max(hi, (P >> 5) + 2);
                    xd::deposit_double(acc, bv);
                }
            }
        }
    }
    lo = xd::row_min_i(lo);
    hi = xr_row_max(hi);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    double v = 0.0;
    if (gl == 0 && row >= 0) v = xd::round_chunks((long long*)acc, *flag, lo, min(hi, xd::NCH - 1));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    // clear what the row touched (the rounding's carries stop at most one chunk above hi)
    if (lo <= hi)
        for (int c = lo + gl; c <= min(hi + 2, xd::NCH - 1); c += XR_GROUP) acc[c] = 0ull;
    if (gl == 0) *flag = 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    return v;
}

// ---- fast path: the row's exact sum in a window of registers.
// A row whose products (and b_i) all start within 4 chunks of each other -- the common
// case: a row's entries and x values span less than ~2^96 -- fits a window of XW = 8 chunks
// [cb, cb + 8) held as int64 (32-bit digits plus carry headroom; the top chunk keeps any
// excess).  The lane accumulates there and rounds it itself; other rows take the 16-lane
// LDS path above.  A row with a non-finite product needs no sum: the flags decide.
constexpr int XW = 8;

__device__ __forceinline__ void xw_add_pieces(long long (&w)[XW], int o, uint64_t p0, uint64_t p1, uint64_t p2,
                                              uint64_t p3, uint64_t p4, bool neg) {
    const long long q[5] = {(long long)p0, (long long)p1, (long long)p2, (long long)p3, (long long)p4};
#pragma unroll
    for (int j = 0; j < XW; ++j) {
        long long add = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t) add += (j == o + t) ? q[t] : 0;
        w[j] += neg ? -add : add;
    }
}

// Exact product a * x (finite, non-zero) into the window at chunk offset o = c - cb.
__device__ __forceinline__ void xw_add_product(long long (&w)[XW], int cb, double a, double x) {
    uint64_t ma, mx;
    int Pa, Px;
    bool na, nx;
    xd::decompose(a, ma, Pa, na);
    xd::decompose(x, mx, Px, nx);
    const uint64_t lo = ma * mx, hi = __umul64hi(ma, mx);
    const int P = Pa + Px - xd::BIAS, c = P >> 5, sh = P & 31;
    const uint64_t w0 = lo << sh;
    const uint64_t w1 = sh ? ((hi << sh) | (lo >> (64 - sh))) : hi;
    const uint64_t w2 = sh ? (hi >> (64 - sh)) : 0;
    xw_add_pieces(w, c - cb, w0 & 0xffffffffull, w0 >> 32, w1 & 0xffffffffull, w1 >> 32, w2, na != nx);
}

// Exact double v (finite, non-zero) into the window.
__device__ __forceinline__ void xw_add_double(long long (&w)[XW], int cb, double v) {
    uint64_t m;
    int P;
    bool neg;
    xd::decompose(v, m, P, neg);
    const int c = P >> 5, sh = P & 31;
    const uint64_t lo = m << sh, hi = sh ? (m >> (64 - sh)) : 0;
    xw_add_pieces(w, c - cb, lo & 0xffffffffull, lo >> 32, hi, 0, 0, neg);
}

__device__ __forceinline__ long long xw_get(const long long (&w)[XW], int j) {
    long long v = 0;
#pragma unroll
    for (int i = 0; i < XW; ++i) v = (i == j) ? w[i] : v;
    return v;
}

// RN_even of sum_j w[j] 2^(32 (cb + j) - BIAS): the exact dot's rounding (round_chunks) on a
// window of registers, every index resolved by unrolled selects.
__device__ __forceinline__ double xw_round(long long (&w)[XW], int cb) {
    long long carry = 0;
#pragma unroll
    for (int j = 0; j < XW; ++j) {           // balanced digits in [-2^31, 2^31)
        const long long v = w[j] + carry;
        if (j < XW - 1) {
            const long long d = (long long)(int32_t)(uint32_t)v;
            carry = (v - d) >> 32;
            w[j] = d;
        } else {
            w[j] = v;
        }
    }
    int top = -1;
#pragma unroll
    for (int j = 0; j < XW; ++j) top = (w[j] != 0) ? j : top;
    if (top < 0) return 0.0;                 // exact zero -> +0
    const bool neg = xw_get(w, top) < 0;
    carry = 0;
#pragma unroll
    for (int j = 0; j < XW; ++j) {           // magnitude in digits [0, 2^32)
        const long long v = (neg ? -w[j] : w[j]) + carry;
        if (j < XW - 1) {
            const long long d = v & 0xffffffffll;
            carry = (v - d) >> 32;
            w[j] = d;
        } else {
            w[j] = v;
        }
    }
    int h = -1;
#pragma unroll
    for (int j = 0; j < XW; ++j) h = (w[j] != 0) ? j : h;
    const uint64_t sign = neg ? 0x8000000000000000ull : 0ull;
    const long long wh = xw_get(w, h);
    // the top chunk may exceed 32 bits (the window's excess)
    const int hb = 63 - __clzll((unsigned long long)wh);
    const int msb = 32 * (cb + h) + hb;
    if (msb >= 2 * xd::BIAS + 1) return __longlong_as_double((long long)(sign | 0x7ff0000000000000ull));   // >= 2^1025
    const int cut = max(msb - 52, 1074);
    // bits [off, off + 64) of the magnitude
    auto dig = [&](int k) -> uint64_t {
        const int j = k - cb;
        return (j >= 0 && j < XW) ? (uint64_t)xw_get(w, j) : 0ull;
    };
    auto get64 = [&](int off) -> uint64_t {
        const int k = off >> 5, sh = off & 31;
        // a digit below the top is < 2^32; the top one may be wider (its high part counts)
        const uint64_t d0 = dig(k), d1 = dig(k + 1), d2 = dig(k + 2);
        uint64_t r = (d0 >> sh) + (d1 << (32 - sh));
        if (sh) r += d2 << (64 - sh);
        else r += d2 << 32 << 32;
        return r;
    };
    const uint64_t mant = get64(cut) & ((1ull << 53) - 1);
    const int g = cut - 1;
    const uint64_t guard = get64(g) & 1ull;
    bool sticky = false;
    {
        const int k = g >> 5, sh = g & 31;
#pragma unroll
        for (int j = 0; j < XW; ++j) sticky |= (cb + j < k) && (w[j] != 0);
        if (sh) sticky |= (dig(k) & ((1ull << sh) - 1)) != 0;
    }
    uint64_t bits = ((uint64_t)(cut - 1074) << 52) + mant;
    if (guard && (sticky || (mant & 1ull))) bits += 1;
    if (bits >= 0x7ff0000000000000ull) bits = 0x7ff0000000000000ull;
    return __longlong_as_double((long long)(sign | bits));
}

// Fast path for one row, one lane per row.  The lane's first XR_HELD entries are loaded
// together and held in registers.  Pass 1 finds the chunks the row's terms start in and
// its non-finite flags; pass 2 sums the terms into the window at the lowest of those
// chunks (entries past the held ones are read again) and the lane rounds it.  Returns
// false when the terms span more than the window (the row then takes the LDS path);
// otherwise v is the rounded value.
constexpr int XR_HELD = 4;

template <bool RESID>
__device__ __forceinline__ void xr_scan(double av, double xv, uint32_t& fl, int& cmin, int& cmax) {
    if (!(isfinite(av) && isfinite(xv))) {
        const double sa = RESID ? -av : av;
        if (isnan(sa) || isnan(xv) || sa == 0.0 || xv == 0.0) fl |= xd::F_NAN;
        else fl |= ((sa > 0.0) == (xv > 0.0)) ? xd::F_PINF : xd::F_NINF;
    } else if (av != 0.0 && xv != 0.0) {
        uint64_t m;
        int Pa, Px;
        bool ng;
        xd::decompose(av, m, Pa, ng);
        xd::decompose(xv, m, Px, ng);
        const int c = (Pa + Px - xd::BIAS) >> 5;
        cmin = min(cmin, c);
        cmax = max(cmax, c);
    }
}

template <class VT, bool RESID>
__device__ __forceinline__ bool exact_row_fast(int row, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, const VT* __restrict__ val,
                                               const double* __restrict__ x, const double* __restrict__ b,
                                               double& v) {
    const int a = rp[row], e = rp[row + 1];
    // the first XR_HELD entries: all loads in flight together
    double ha[XR_HELD], hx[XR_HELD];
    int32_t hc[XR_HELD];
#pragma unroll
    for (int i = 0; i < XR_HELD; ++i) {
        hc[i] = 0;
        ha[i] = 0.0;
        if (a + i < e) {
            hc[i] = ci[a + i];
            ha[i] = (double)val[a + i];
        }
    }
#pragma unroll
    for (int i = 0; i < XR_HELD; ++i) hx[i] = x[hc[i]];       // an unused slot reads x[0]
    uint32_t fl = 0;
    int cmin = INT_MAX, cmax = INT_MIN;
#pragma unroll
    for (int i = 0; i < XR_HELD; ++i) {
        if (a + i < e) xr_scan<RESID>(ha[i], hx[i], fl, cmin, cmax);
    }
    for (int k = a + XR_HELD; k < e; ++k) xr_scan<RESID>((double)val[k], x[ci[k]], fl, cmin, cmax);
    double bv = 0.0;
    if constexpr (RESID) {
        bv = b[row];
        if (!isfinite(bv)) {
            if (isnan(bv)) fl |= xd::F_NAN;
            else fl |= bv > 0.0 ? xd::F_PINF : xd::F_NINF;
        } else if (bv != 0.0) {
            uint64_t m;
            int P;
            bool ng;
            xd::decompose(bv, m, P, ng);
            cmin = min(cmin, P >> 5);
            cmax = max(cmax, P >> 5);
        }
    }
    if (fl) {
        if ((fl & xd::F_NAN) || ((fl & xd::F_PINF) && (fl & xd::F_NINF))) v = __longlong_as_double(0x7ff8000000000000ll);
        else v = (fl & xd::F_PINF) ? __longlong_as_double(0x7ff0000000000000ll)
                                   : __longlong_as_double((long long)0xfff0000000000000ull);
        return true;
    }
    if (cmin > cmax) {              // no non-zero term
        v = 0.0;
        return true;
    }
    if (cmax - cmin > XW - 5) return false;
    long long w[XW];
#pragma unroll
    for (int j = 0; j < XW; ++j) w[j] = 0;
#pragma unroll
    for (int i = 0; i < XR_HELD; ++i) {
        if (ha[i] != 0.0 && hx[i] != 0.0) xw_add_product(w, cmin, RESID ? -ha[i] : ha[i], hx[i]);
    }
    for (int k = a + XR_HELD; k < e; ++k) {
        const double av = (double)val[k], xv = x[ci[k]];
        if (av != 0.0 && xv != 0.0) xw_add_product(w, cmin, RESID ? -av : av, xv);
    }
    if constexpr (RESID) {
        if (bv != 0.0) xw_add_double(w, cmin, bv);
    }
    v = xw_round(w, cmin);
    return true;
}

// The same from the offset form of A (slice c = the row's 256-row slice, t its lane): the
// row's value slots (unit-stride across the slice), its mask byte and the slice's offsets,
// all loaded together; every term is held (at most OFS_MAX), none is read twice.
template <class VT, bool RESID>
__device__ __forceinline__ bool exact_row_fast_ofs(int row, int c, int t, const Sliced<VT>& sl,
                                                   const double* __restrict__ x, const double* __restrict__ b,
                                                   double& v) {
    const int64_t base = sl.off[c];
    const int K = (int)((sl.off[c + 1] - base) / 256);
    const uint32_t m = sl.mask[row];
    double ha[OFS_MAX], hx[OFS_MAX];
    int hc[OFS_MAX];
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) {
        ha[j] = 0.0;
        hc[j] = 0;
        if (j < K) {
            ha[j] = (double)sl.val[base + (int64_t)j * 256 + t];
            if ((m >> j) & 1u) hc[j] = row + sl.ofs[(int64_t)c * OFS_MAX + j];
        }
    }
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) hx[j] = x[hc[j]];       // an unmarked slot reads x[0]
    uint32_t fl = 0;
    int cmin = INT_MAX, cmax = INT_MIN;
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) {
        if ((m >> j) & 1u) xr_scan<RESID>(ha[j], hx[j], fl, cmin, cmax);
    }
    double bv = 0.0;
    if constexpr (RESID) {
        bv = b[row];
        if (!isfinite(bv)) {
            if (isnan(bv)) fl |= xd::F_NAN;
            else fl |= bv > 0.0 ? xd::F_PINF : xd::F_NINF;
        } else if (bv != 0.0) {
            uint64_t mb;
            int P;
            bool ng;
            xd::decompose(bv, mb, P, ng);
            cmin = min(cmin, P >> 5);
            cmax = max(cmax, P >> 5);
        }
    }
    if (fl) {
        if ((fl & xd::F_NAN) || ((fl & xd::F_PINF) && (fl & xd::F_NINF))) v = __longlong_as_double(0x7ff8000000000000ll);
        else v = (fl & xd::F_PINF) ? __longlong_as_double(0x7ff0000000000000ll)
                                   : __longlong_as_double((long long)0xfff0000000000000ull);
        return true;
    }
    if (cmin > cmax) {
        v = 0.0;
        return true;
    }
    if (cmax - cmin > XW - 5) return false;
    long long w[XW];
#pragma unroll
    for (int j = 0; j < XW; ++j) w[j] = 0;
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) {
        if (((m >> j) & 1u) && ha[j] != 0.0 && hx[j] != 0.0) xw_add_product(w, cmin, RESID ? -ha[j] : ha[j], hx[j]);
    }
    if constexpr (RESID) {
        if (bv != 0.0) xw_add_double(w, cmin, bv);
    }
    v = xw_round(w, cmin);
    return true;
}

// One chunk of 256 rows for a block of 256 threads: each lane its own row on the fast
// path (OFS: read from the offset form sl, whose slices are these chunks), then the rows
// that need the LDS path in groups of 16 lanes (read from CSR); `out(row, value)` for
// every row of the chunk.  accs / flags: the LDS path's accumulators (zero), list: 256
// ints, count: two ints used alternately (parity = the block's chunk counter; both zero
// before the first chunk).  Block-uniform.
template <class VT, bool RESID, bool OFS, class Out>
__device__ __forceinline__ void exact_rows_chunk(int r0, int n, int parity, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const VT* __restrict__ val,
                                                 const double* __restrict__ x, const double* __restrict__ b,
                                                 const Sliced<VT>& sl, unsigned long long* accs, uint32_t* flags,
                                                 int* list, int* count, Out& out) {
    const int t = threadIdx.x, row = r0 + t;
    if (row < n) {
        double v;
        bool done;
        if constexpr (OFS) done = exact_row_fast_ofs<VT, RESID>(row, r0 / 256, t, sl, x, b, v);
        else done = exact_row_fast<VT, RESID>(row, rp, ci, val, x, b, v);
        if (done) out(row, v);
        else list[atomicAdd(&count[parity], 1)] = row;
    }
    __syncthreads();
    const int m = count[parity];
    // the other counter was last read before this chunk's barrier; the next chunk uses it
    // only after the closing barrier below
    if (t == 0) count[parity ^ 1] = 0;
    const int g = t / XR_GROUP, gl = t % XR_GROUP;
    for (int j0 = 0; j0 < m; j0 += XR_ROWS) {     // uniform over the block
        const int j = j0 + g;
        const int srow = j < m ? list[j] : -1;
        const double v = exact_row<VT, RESID>(srow, rp, ci, val, x, b, accs + g * xd::NCH, flags + g, gl);
        if (gl == 0 && srow >= 0) out(srow, v);
    }
    __syncthreads();
}

// Every row of the block's steps of XR_ROWS rows on the LDS path (FAST = false: the
// matrices whose rows are long).
template <class VT, bool RESID, class Out>
__device__ __forceinline__ void exact_rows_lds(int n, int first, int stride, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, const VT* __restrict__ val,
                                               const double* __restrict__ x, const double* __restrict__ b,
                                               unsigned long long* accs, uint32_t* flags, Out& out) {
    const int g = threadIdx.x / XR_GROUP, gl = threadIdx.x % XR_GROUP;
    const int steps = (n + XR_ROWS - 1) / XR_ROWS;
    for (int st = first; st < steps; st += stride) {   // uniform over the block
        const int row = st * XR_ROWS + g;
        const double v = exact_row<VT, RESID>(row < n ? row : -1, rp, ci, val, x, b, accs + g * xd::NCH,
                                               flags + g, gl);
        if (gl == 0 && row < n) out(row, v);
    }
}

template <class Epi>
struct XrStore {
    Epi& epi;
    __device__ __forceinline__ void operator()(int row, double v) { epi(row, v); }
};

// y = A x with exactly rounded rows (RESID: r = b - A x, each row rounded once), epilogue
// epi(row, value); block 0 may carry a finalize role.  FAST: the one-lane-per-row register
// path first (short rows), else every row on the LDS path.
template <class VT, class Epi, class Fin, bool RESID, bool FAST, bool OFS = false>
__global__ void __launch_bounds__(256)
spmv_exact_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                  const VT* __restrict__ val, const double* __restrict__ x, const double* __restrict__ b,
                  Epi epi, Fin fin, const int* halt, Sliced<VT> sl) {
    if (halt && *halt) return;
    constexpr int XS = XR_SMEM + (FAST ? 256 * 4 + 16 : 0);
    constexpr int SMEM = Fin::SMEM > XS ? Fin::SMEM : XS;
    __shared__ __align__(16) unsigned char smem[SMEM];
    int bfirst = 0;
    if constexpr (Fin::D > 0) {
        if (blockIdx.x == 0) {
            fin.run(smem);
            return;
        }
        bfirst = 1;
    }
    unsigned long long* accs = (unsigned long long*)smem;
    uint32_t* flags = (uint32_t*)(smem + XR_ROWS * xd::NCH * 8);
    int* list = (int*)(smem + XR_SMEM);
    int* count = list + 256;
    for (int i = threadIdx.x; i < XR_ROWS * xd::NCH; i += blockDim.x) accs[i] = 0ull;
    if (threadIdx.x < XR_ROWS) flags[threadIdx.x] = 0u;
    if (FAST && threadIdx.x < 2) count[threadIdx.x] = 0;
    __syncthreads();
    XrStore<Epi> out{epi};
    const int G = (int)gridDim.x - bfirst;
    if constexpr (FAST) {
        const int nchunk = (n + 255) / 256;
        int parity = 0;
        for (int c = (int)blockIdx.x - bfirst; c < nchunk; c += G, parity ^= 1)
            exact_rows_chunk<VT, RESID, OFS>(c * 256, n, parity, rp, ci, val, x, b, sl, accs, flags, list, count,
                                             out);
    } else {
        exact_rows_lds<VT, RESID>(n, (int)blockIdx.x - bfirst, G, rp, ci, val, x, b, accs, flags, out);
    }
}

template <int D, int K, class Epi>
struct XrDot {
    Epi& epi;
    double (&e)[D][K];
    unsigned long long* acc;
    uint32_t* fl;
    __device__ __forceinline__ void operator()(int row, double v) {
        double xa[D], ya[D];
        epi.row(row, v, xa, ya);
#pragma unroll
        for (int d = 0; d < D; ++d) xd::accumulate<K>(e[d], xa[d], ya[d], acc + d * xd::NCH, &fl[d]);
    }
};

// The same with D exact dots of the rows' values in the epilogue (the true residual and
// its norm): epi.row(row, value, xa, ya) as in the row-sequential dot kernels.
template <int D, int K, class VT, class Epi, bool RESID, bool FAST, bool OFS = false>
__global__ void __launch_bounds__(256)
spmv_exact_dot_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                      const VT* __restrict__ val, const double* __restrict__ x, const double* __restrict__ b,
                      Epi epi, xd::Site site, const int* halt, Sliced<VT> sl) {
    if (halt && *halt) return;
    XD_SHARED(D)
    __shared__ __align__(16) unsigned char smem[XR_SMEM + (FAST ? 256 * 4 + 16 : 0)];
    xd::block_init<D>(sh_acc, sh_flags);
    epi.load();
    unsigned long long* accs = (unsigned long long*)smem;
    uint32_t* flags = (uint32_t*)(smem + XR_ROWS * xd::NCH * 8);
    int* list = (int*)(smem + XR_SMEM);
    int* count = list + 256;
    for (int i = threadIdx.x; i < XR_ROWS * xd::NCH; i += blockDim.x) accs[i] = 0ull;
    if (threadIdx.x < XR_ROWS) flags[threadIdx.x] = 0u;
    if (FAST && threadIdx.x < 2) count[threadIdx.x] = 0;
    __syncthreads();
    double e[D][K];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k = 0; k < K; ++k) e[d][k] = 0.0;
    XrDot<D, K, Epi> out{epi, e, sh_acc, sh_flags};
    if constexpr (FAST) {
        const int nchunk = (n + 255) / 256;
        int parity = 0;
        for (int c = blockIdx.x; c < nchunk; c += gridDim.x, parity ^= 1)
            exact_rows_chunk<VT, RESID, OFS>(c * 256, n, parity, rp, ci, val, x, b, sl, accs, flags, list, count,
                                             out);
    } else {
        exact_rows_lds<VT, RESID>(n, blockIdx.x, gridDim.x, rp, ci, val, x, b, accs, flags, out);
    }
    __syncthreads();
    xd::block_flush<D, K>(e, sh_acc);
    xd::block_write<D>(site, sh_acc, sh_flags, sh_tmp, sh_rng);
}

// epilogues taking the exactly rounded residual row r (not A x)
template <class T>
struct EpiResidX {          // r (and copies c1, c2 at initialisation)
    T* r;
    T* c1;
    T* c2;
    __device__ __forceinline__ void operator()(int row, T v) const {
        r[row] = v;
        if (c1) c1[row] = v;
        if (c2) c2[row] = v;
    }
};
template <class Fin>
struct EpiResidXDot {       // r and the dot (r, r)
    double* res;
    Fin fin;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void row(int i, double v, double (&xa)[1], double (&ya)[1]) {
        res[i] = v;
        xa[0] = v;
        ya[0] = v;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

}  // namespace pbcg
