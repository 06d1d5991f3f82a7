// HIP kernels of the p-BiCGStab hot path (gfx950, wave64).
//
//  * spmv_seq_kernel   row-sequential CSR SpMV: every row is summed left to right by
//                      one lane (the summation order of the plain definition of A.x),
//                      with the block's val/col range staged through LDS by coalesced
//                      loads in chunks; XCD-aware block -> row-range mapping.  SL: the
//                      same sums read from a sliced (column-major, 256-row slice) copy.
//  * spmv_kernel       vector-CSR SpMV: L lanes per row (L = 2..32 from the mean row
//                      length, or L = 64: one wavefront per row), coalesced val/col
//                      reads, xor-butterfly row reduction (same bits in every lane).
//  * spmv_*dot_kernel  the same row loops, persistent grid, with an epilogue that
//                      produces D exact dot products (BiCGStab, true residual).
//  * ew_dot_kernel     one fused element-wise pass (vector updates) with D exact dot
//                      products accumulated on the fly (p-BiCGStab phases A and B).
//  * ew_fdot_kernel    the FP32 analogue with plain FP32 dot products reduced in a
//                      fixed tree (the inner solver of the refinement driver).
// Every arithmetic expression is written in the parenthesisation of the paper's
// recurrences and compiled without contraction.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <limits.h>
#include <stdint.h>

#include <type_traits>

#include "state.hpp"
#include "xdot.hpp"

#pragma clang fp contract(off)

namespace pbcg {

constexpr int NUM_XCD = 8;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring rows share an L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    int xcd = b % NUM_XCD, idx = b / NUM_XCD;
    int base = G / NUM_XCD, rem = G % NUM_XCD;
    return xcd * base + min(xcd, rem) + idx;
}

// per-block partials of a plain-dot site (T = float for the FP32 solver, double for
// the ordinary-dot FP64 comparator)
template <class T>
struct TSite {
    T* part;                // [grid][D]
};
using FSite = TSite<float>;

// Fixed-order tree over the G per-block partials (blockDim.x == 256).
template <int D, class T>
__device__ void fdot_reduce(const TSite<T>& site, int G, T* sh /* D*256 */, T* res /* D */) {
    const int t = threadIdx.x;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        T s = T(0);
        for (int g = t; g < G; g += 256) s = s + site.part[(size_t)g * D + d];
        sh[d * 256 + t] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int d = 0; d < D; ++d) sh[d * 256 + t] = sh[d * 256 + t] + sh[d * 256 + t + w];
        }
        __syncthreads();
    }
    if (t < D) res[t] = sh[t * 256];
    __syncthreads();
}

// "Finalize roles": the cross-block reduction of a dot site plus the scalar work that
// follows it, run by one 256-thread block -- either a block of its own kernel, or block 0
// of the next kernel in the stream when that kernel does not consume the results (the
// SpMV after each p-BiCGStab phase), which hides its latency behind the SpMV.
constexpr int DOT_GMAX = 1024;

struct NoFin {
    static constexpr int D = 0;
    static constexpr int SMEM = 0;
    __device__ void run(unsigned char*) {}
};

// GM: the largest producer grid the role accepts (sizes its LDS)
template <int D_, class Op, int GM = DOT_GMAX>
struct XFin {                       // exact dots
    static constexpr int D = D_;
    static constexpr int BLOCK = 1024;  // threads of its own kernel (any count works)
    static constexpr int SMEM = 32 + 4 * xd::NCH * 8 + 16 + 32 + 2 * GM * 4 * 2;
    Op op;
    xd::Site site;
    int G;
    const int* halt;
    __device__ void run(unsigned char* smem) {
        if (halt && *halt) return;
        double* res = (double*)smem;                              // 4 doubles
        long long* fin = (long long*)(smem + 32);                 // D*NCH
        uint32_t* fl = (uint32_t*)(smem + 32 + 4 * xd::NCH * 8);  // 4
        int* rng = (int*)(fl + 4);                                // 8
        short* hlo = (short*)(rng + 8);                           // GM*4
        short* hhi = hlo + GM * 4;
        xd::reduce_records<D, GM>(site, G, fin, hlo, hhi, fl, rng, res);
        if (threadIdx.x == 0) op.finalize(res);
    }
};

template <class T, int D_, class Op>
struct TFin {                       // plain dots in a fixed tree
    static constexpr int D = D_;
    static constexpr int BLOCK = 256;   // the tree is defined for 256 threads
    static constexpr int SMEM = (4 + 4 * 256) * (int)sizeof(T);
    Op op;
    TSite<T> site;
    int G;
    const int* halt;
    __device__ void run(unsigned char* smem) {
        if (halt && *halt) return;
        T* res = (T*)smem;
        T* sh = res + 4;
        fdot_reduce<D>(site, G, sh, res);
        if (threadIdx.x == 0) op.finalize(res);
    }
};
template <int D, class Op>
using FFin = TFin<float, D, Op>;

template <class Fin>
__global__ void __launch_bounds__(Fin::BLOCK) fin_kernel(Fin fin) {
    __shared__ __align__(16) unsigned char smem[Fin::SMEM];
    fin.run(smem);
}

// ----------------------------------------------------------------------------- SpMV
template <class T>
struct EpiStore {
    T* y;
    __device__ __forceinline__ void operator()(int row, T s) const { y[row] = s; }
};

// r = b - A x; optional copies into c1, c2 (r_hat, p at initialisation)
template <class T>
struct EpiResid {
    const T* b;
    T* r;
    T* c1;
    T* c2;
    __device__ __forceinline__ void operator()(int row, T s) const {
        T v = b[row] - s;
        r[row] = v;
        if (c1) c1[row] = v;
        if (c2) c2[row] = v;
    }
};

template <int L, class VT, class XT, class AT, class Epi>
__global__ void __launch_bounds__(256)
spmv_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
            const VT* __restrict__ val, const XT* __restrict__ x, Epi epi, const int* halt) {
    if (halt && *halt) return;
    const int rows_per_block = blockDim.x / L;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int row = blk * rows_per_block + (int)threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= n) return;  // whole L-lane groups exit together
    const int a = rp[row], b = rp[row + 1];
    AT s = AT(0);
    for (int k = a + lane; k < b; k += L) {
        AT prod = (AT)val[k] * (AT)x[ci[k]];
        s = s + prod;
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) s = s + __shfl_xor(s, o);
    if (lane == 0) epi(row, s);
}

// Sliced copy of a CSR matrix (built by slice_width/scan/fill below): slice c holds rows
// 256c .. 256c+255 column-major, entry k of the row in lane t at off[c] + 256 k + t,
// padded to the slice's longest row (padding: col 0, value 0, never read for arithmetic).
template <class VT>
struct Sliced {
    const int64_t* off = nullptr;   // [nslice + 1] entry offsets; null: use the CSR arrays
    const int32_t* col = nullptr;   // 32-bit columns, or (SL_D16) 16-bit residuals
    const VT* val = nullptr;
    const int32_t* base = nullptr;  // SL_D16: per slice and position, at off[c] / 256 + k
    const int32_t* perm = nullptr;  // SL_PERM: the row held by each slot (slice height 64)
    const uint8_t* mask = nullptr;  // SL_OFS: per row, bit j set when the row has column row + d_j
    const int32_t* ofs = nullptr;   // SL_OFS: per slice, the offsets d_0 < d_1 < ... (OFS_MAX slots)
};

constexpr int SLICE_UNROLL = 8;   // entries of a row loaded ahead of their additions
static_assert(64 % SLICE_UNROLL == 0, "the base broadcast covers whole unrolled steps");

// One lane's row of slice c of a sliced copy (len entries, storage order): s (and the
// Dot2 compensation cmp when COMP) accumulate exactly as in the staged path below.
// Layout flags SLF of a sliced copy: SL_NT -- the slice's values and column entries are read
// with non-temporal loads (a matrix larger than the Infinity Cache streams past it instead
// of evicting the vectors); SL_D16 -- entry k of row r in slice c stores the 16-bit residual
// col - r - base[c][k], where base[c][k] is the smallest col - r at position k over the
// slice's rows (every residual of the matrix fits in 16 bits): two bytes per entry less
// than 32-bit columns.  On a stencil each position holds one or two neighbour offsets.
constexpr int SL_NT = 1, SL_D16 = 2;
// SL_PERM: the row-sorted copy for matrices of irregular row lengths (random sparsity):
// slices of 64 rows (one wavefront), the rows of each window of WSORT consecutive rows
// ordered by decreasing length (ties: ascending row) so that a slice holds rows of nearly
// equal length; slot j of the order holds row perm[j], and entry k of slot 64c + t sits at
// off[c] + 64 k + t.  Each lane still sums its own row left to right in storage order.
constexpr int SL_PERM = 4;
constexpr int WS_ROWS = 64;
constexpr int WSORT = 4096;
// SL_OFS: the offset form for banded and stencil matrices, where the rows of a slice draw
// their columns from at most OFS_MAX offsets col - row.  Slice c lists its offsets
// d_0 < ... < d_{K-1} once; slot j of row r holds the value of entry (r, r + d_j), or 0 when
// the row has no such entry, and bit j of the row's mask byte says which slots exist.  No
// column entries are stored: per row, K values and one byte against K values and K column
// entries (and the row pointers) of the other forms.  Columns ascend within a row, so the
// slots' order is the row's storage order and the lane adds the same products in the same
// order (missing slots are skipped, never added).
constexpr int SL_OFS = 8;
constexpr int OFS_MAX = 8;

template <class VT, class XT, class AT, bool COMP, int SLF = 0>
__device__ __forceinline__ void slice_row(const Sliced<VT>& sl, int c, int t, int len, const XT* __restrict__ x,
                                          AT& s, AT& cmp) {
    constexpr int U = SLICE_UNROLL, R = 256;
    constexpr bool MNT = (SLF & SL_NT) != 0, D16 = (SLF & SL_D16) != 0;
    const int64_t base = sl.off[c];
    const int w = (int)((sl.off[c + 1] - base) / R);
    const int row = c * R + t;
    const VT* __restrict__ vp = sl.val + base + t;
    const int32_t* __restrict__ cp = sl.col + base + t;
    const uint16_t* __restrict__ dp = (const uint16_t*)sl.col + base + t;
    const int32_t* __restrict__ bp = sl.base + base / R;
    int bv = 0;   // D16: bases of positions 64j .. 64j + 63, lane l holding position 64j + l
    for (int k0 = 0; k0 < w; k0 += U) {
        if constexpr (D16) {
            if ((k0 & 63) == 0) {   // one coalesced load per 64 positions (U divides 64)
                const int kk = k0 + (threadIdx.x & 63);
                bv = kk < w ? bp[kk] : 0;
            }
        }
        VT av[U];
        int32_t cv[U];
        // all loads of the step are issued before any of them is used
#pragma unroll
        for (int u = 0; u < U; ++u) {
            av[u] = VT(0);
            cv[u] = 0;
            if (k0 + u < w) {
                const int64_t o = (int64_t)(k0 + u) * R;
                if constexpr (MNT) {
                    av[u] = __builtin_nontemporal_load(vp + o);
                    if constexpr (D16) cv[u] = __builtin_nontemporal_load(dp + o);
                    else cv[u] = __builtin_nontemporal_load(cp + o);
                } else {
                    av[u] = vp[o];
                    if constexpr (D16) cv[u] = dp[o];
                    else cv[u] = cp[o];
                }
            }
        }
        if constexpr (D16) {   // residual -> column
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k0 + u < w) cv[u] += row + __builtin_amdgcn_readlane(bv, (k0 + u) & 63);
        }
        // gathers without branches (an entry past the row end reads x[0] and is not added),
        // so that all U gathers are in flight together
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[(k0 + u < len) ? cv[u] : 0];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u < len) {
                const AT a = (AT)av[u], xx = (AT)xv[u];
                const AT prod = a * xx;
                if constexpr (COMP) {
                    const float pe = fmaf(a, xx, -prod);
                    const float sn = s + prod;
                    const float bb = sn - s;
                    const float err = (s - (sn - bb)) + (prod - bb);
                    s = sn;
                    cmp = cmp + (err + pe);
                } else {
                    s = s + prod;
                }
            }
        }
    }
}

// One lane's row of slice c of an offset-form copy (SL_OFS): the K slot values of the row
// (unit-stride across the slice), the x gathers of the slots the mask marks (unmarked slots
// read x[0] and are not added), the additions in slot order.
template <class VT, class XT, class AT, bool COMP, int SLF>
__device__ __forceinline__ void slice_row_ofs(const Sliced<VT>& sl, int c, int t, const XT* __restrict__ x,
                                              AT& s, AT& cmp) {
    constexpr int R = 256;
    constexpr bool MNT = (SLF & SL_NT) != 0;
    const int64_t base = sl.off[c];
    const int K = (int)((sl.off[c + 1] - base) / R);
    const int row = c * R + t;
    const uint32_t m = MNT ? (uint32_t)__builtin_nontemporal_load(sl.mask + row) : (uint32_t)sl.mask[row];
    const int dl = sl.ofs[(int64_t)c * OFS_MAX + (threadIdx.x & (OFS_MAX - 1))];   // lane l: d_(l mod 8)
    const VT* __restrict__ vp = sl.val + base + t;
    VT av[OFS_MAX];
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) {
        av[j] = VT(0);
        if (j < K) av[j] = MNT ? __builtin_nontemporal_load(vp + (int64_t)j * R) : vp[(int64_t)j * R];
    }
    XT xv[OFS_MAX];
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) xv[j] = x[((m >> j) & 1u) ? row + __builtin_amdgcn_readlane(dl, j) : 0];
#pragma unroll
    for (int j = 0; j < OFS_MAX; ++j) {
        if ((m >> j) & 1u) {
            const AT a = (AT)av[j], xx = (AT)xv[j];
            const AT prod = a * xx;
            if constexpr (COMP) {
                const float pe = fmaf(a, xx, -prod);
                const float sn = s + prod;
                const float bb = sn - s;
                const float err = (s - (sn - bb)) + (prod - bb);
                s = sn;
                cmp = cmp + (err + pe);
            } else {
                s = s + prod;
            }
        }
    }
}

// One lane's row (len entries) in wave slice ws of a row-sorted copy.  Loads are masked by
// the row's own length, so a slice's padding is never fetched; the x gathers are issued
// without branches (a slot past the row end reads x[0] and is not added).
template <class VT, class XT, class AT, bool COMP, int SLF>
__device__ __forceinline__ void wslice_row(const Sliced<VT>& sl, int ws, int lane, int len,
                                           const XT* __restrict__ x, AT& s, AT& cmp) {
    constexpr int U = SLICE_UNROLL, R = WS_ROWS;
    constexpr bool MNT = (SLF & SL_NT) != 0;
    const int64_t base = sl.off[ws];
    const int w = (int)((sl.off[ws + 1] - base) / R);
    const VT* __restrict__ vp = sl.val + base + lane;
    const int32_t* __restrict__ cp = sl.col + base + lane;
    for (int k0 = 0; k0 < w; k0 += U) {
        VT av[U];
        int32_t cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            av[u] = VT(0);
            cv[u] = 0;
            if (k0 + u < len) {
                const int64_t o = (int64_t)(k0 + u) * R;
                if constexpr (MNT) {
                    av[u] = __builtin_nontemporal_load(vp + o);
                    cv[u] = __builtin_nontemporal_load(cp + o);
                } else {
                    av[u] = vp[o];
                    cv[u] = cp[o];
                }
            }
        }
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[cv[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u < len) {
                const AT a = (AT)av[u], xx = (AT)xv[u];
                const AT prod = a * xx;
                if constexpr (COMP) {
                    const float pe = fmaf(a, xx, -prod);
                    const float sn = s + prod;
                    const float bb = sn - s;
                    const float err = (s - (sn - bb)) + (prod - bb);
                    s = sn;
                    cmp = cmp + (err + pe);
                } else {
                    s = s + prod;
                }
            }
        }
    }
}

// Row-sequential SpMV engine (persistent, product-staged).
//
// Rows are taken in chunks of R = blockDim.x rows, one row per lane, and every row is
// summed left to right in storage order.  The chunk's nonzeros are swept in windows of
// CAP entries: all lanes read val/col of the window with unit-stride (coalesced) loads,
// gather x, and park the rounded products a_k * x_col(k) in LDS; after a barrier each
// lane adds the products of its own row that fall in the window, carrying its running
// sum into the next window.  The additions therefore happen in storage order whatever
// the row lengths (a row longer than CAP simply spans several windows), and the gathers
// of a whole window are in flight together instead of one per lane and step.
// Chunks are dealt to the worker blocks of each XCD from a contiguous range of rows
// (hardware block b runs on XCD b % 8), so the x planes a stencil row touches are
// shared in that XCD's L2.
//
// With a sliced copy (SL, view in sl) a chunk is one slice: each lane walks its own row with
// unit-stride (coalesced) val/col loads across the slice and gathers x for the entries
// of its row; no LDS and no barriers.  Neighbouring lanes hold neighbouring rows, so
// a stencil's gathers of one entry position are coalesced as well.  The additions are
// the same as in the staged path (storage order), so the results are bit-identical.
//
// COMP (float only): compensated accumulation, algorithm Dot2 of Ogita, Rump and Oishi
// (2005) in storage order -- the window holds (p, e) with p = fl(a x) and the exact
// product error e = fma(a, x, -p); each lane runs TwoSum(s, p) and adds err + e into a
// compensation c; the row's value is fl(s + c).  All arithmetic is float32.
template <int CAP, class VT, class XT, class AT, class Body, bool COMP = false, bool SL = false, int SLF = 0>
__device__ __forceinline__ void seq_stage(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                          const VT* __restrict__ val, const XT* __restrict__ x,
                                          int bfirst, int G, AT* sprod, Body& body, Sliced<VT> sl = {}) {
    static_assert(!COMP || (sizeof(AT) == 4 && sizeof(VT) == 4 && sizeof(XT) == 4), "Dot2 path is float32");
    constexpr int R = 256;            // blockDim.x
    constexpr int PER = CAP / R;
    const int nchunk = (n + R - 1) / R;
    const int hb = blockIdx.x;
    int cbeg, cend, gper, bi;
    if (G >= NUM_XCD) {
        const int xcd = hb % NUM_XCD;
        auto cnt = [&](int m) { return (m + NUM_XCD - 1 - xcd) / NUM_XCD; };  // #h in [0,m), h%8==xcd
        gper = cnt(bfirst + G) - cnt(bfirst);
        bi = cnt(hb) - cnt(bfirst);
        cbeg = (int)((long long)nchunk * xcd / NUM_XCD);
        cend = (int)((long long)nchunk * (xcd + 1) / NUM_XCD);
    } else {
        gper = G;
        bi = hb - bfirst;
        cbeg = 0;
        cend = nchunk;
    }
    const int t = threadIdx.x;
    for (int c = cbeg + bi; c < cend; c += gper) {
        if constexpr (SL && (SLF & SL_PERM) != 0) {
            // row-sorted copy: chunk c is wave slices 4c .. 4c + 3 (slots 256c ..)
            const int slot = c * R + t;
            if (slot < n) {
                const int prow = sl.perm[slot];
                const int pa = rp[prow], pb = rp[prow + 1];
                AT s = AT(0), cmp = AT(0);
                wslice_row<VT, XT, AT, COMP, SLF>(sl, slot / WS_ROWS, t % WS_ROWS, pb - pa, x, s, cmp);
                if constexpr (COMP) s = s + cmp;
                body(prow, s);
            }
            continue;
        }
        const int r0 = c * R, r1 = min(r0 + R, n), row = r0 + t;
        if constexpr (SL && (SLF & SL_OFS) != 0) {
            AT s = AT(0), cmp = AT(0);
            slice_row_ofs<VT, XT, AT, COMP, SLF>(sl, c, t, x, s, cmp);
            if constexpr (COMP) s = s + cmp;
            if (row < r1) body(row, s);
            continue;
        }
        int RA = 0, RB = 0;
        if (row < r1) { RA = rp[row]; RB = rp[row + 1]; }
        AT s = AT(0), cmp = AT(0);
        if constexpr (SL) {
            slice_row<VT, XT, AT, COMP, SLF>(sl, c, t, RB - RA, x, s, cmp);
        } else {
            const int A0 = rp[r0], A1 = rp[r1];
            for (int w = A0; w < A1; w += CAP) {
                const int we = min(w + CAP, A1);
                VT pv[PER];
                int32_t pc[PER];
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const int k = w + t + j * R;
                    pv[j] = VT(0);
                    pc[j] = 0;
                    if (k < we) { pv[j] = val[k]; pc[j] = ci[k]; }
                }
                // gathers without branches (a slot past the window reads x[0], unused), so
                // that all PER gathers are in flight together
                XT xg[PER];
#pragma unroll
                for (int j = 0; j < PER; ++j) xg[j] = x[pc[j]];
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const int k = w + t + j * R;
                    if (k < we) {
                        const AT a = (AT)pv[j], xv = (AT)xg[j];
                        AT prod = a * xv;
                        if constexpr (COMP) {
                            float2* sp2 = (float2*)sprod;
                            sp2[k - w] = make_float2(prod, fmaf(a, xv, -prod));
                        } else {
                            sprod[k - w] = prod;
                        }
                    }
                }
                __syncthreads();
                const int ka = max(RA, w), kb = min(RB, we);
                if constexpr (COMP) {
                    const float2* sp2 = (const float2*)sprod;
                    for (int k = ka; k < kb; ++k) {
                        const float2 pe = sp2[k - w];
                        const float sn = s + pe.x;
                        const float bb = sn - s;
                        const float err = (s - (sn - bb)) + (pe.x - bb);
                        s = sn;
                        cmp = cmp + (err + pe.y);
                    }
                } else {
                    for (int k = ka; k < kb; ++k) s = s + sprod[k - w];
                }
                __syncthreads();
            }
        }
        if constexpr (COMP) s = s + cmp;
        if (row < r1) body(row, s);
    }
}

constexpr int SEQ_CAP = 2048;   // staged products per window (8 per lane)

template <class Epi>
struct StoreBody {
    Epi& epi;
    template <class AT>
    __device__ __forceinline__ void operator()(int row, AT s) { epi(row, s); }
};

// grid = worker blocks (+1 when block 0 carries a finalize role)
template <class VT, class XT, class AT, class Epi, class Fin, bool COMP = false, bool SL = false, int SLF = 0>
__global__ void __launch_bounds__(256)
spmv_seq_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                const VT* __restrict__ val, const XT* __restrict__ x, Epi epi, Fin fin, const int* halt,
                Sliced<VT> sl) {
    if (halt && *halt) return;
    constexpr int STAGE = SL ? 16 : SEQ_CAP * (int)sizeof(AT) * (COMP ? 2 : 1);
    constexpr int SMEM = Fin::SMEM > STAGE ? Fin::SMEM : STAGE;
    __shared__ __align__(16) unsigned char smem[SMEM];
    int bfirst = 0;
    if constexpr (Fin::D > 0) {
        if (blockIdx.x == 0) {      // finalize role of the previous kernel's dot site
            fin.run(smem);
            return;
        }
        bfirst = 1;
    }
    StoreBody<Epi> body{epi};
    seq_stage<SEQ_CAP, VT, XT, AT, StoreBody<Epi>, COMP, SL, SLF>(n, rp, ci, val, x, bfirst,
                                                                   (int)gridDim.x - bfirst, (AT*)smem, body, sl);
}

// Sliced copy, step 0: clear the residual-overflow flag (off[nslice + 1]).
__global__ void slice_clear_kernel(int64_t* __restrict__ slot) { *slot = 0; }

// Step 1: off[c + 1] = 256 * (longest row of slice c), off[0] = 0.
__global__ void __launch_bounds__(256) slice_width_kernel(int n, const int32_t* __restrict__ rp,
                                                          int64_t* __restrict__ off) {
    __shared__ int sh[4];
    const int c = blockIdx.x, t = threadIdx.x, row = c * 256 + t;
    int len = row < n ? rp[row + 1] - rp[row] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o));
    if ((t & 63) == 0) sh[t >> 6] = len;
    __syncthreads();
    if (t == 0) {
        off[c + 1] = 256LL * max(max(sh[0], sh[1]), max(sh[2], sh[3]));
        if (c == 0) off[0] = 0;
    }
}

// Step 2 (one block of 1024): off[1..ns] -> inclusive prefix sums.
__global__ void __launch_bounds__(1024) slice_scan_kernel(int ns, int64_t* __restrict__ off) {
    __shared__ int64_t sh[1024];
    const int t = threadIdx.x;
    const int per = (ns + 1023) / 1024;
    const int64_t a = 1 + (int64_t)t * per, b = min(a + per, (int64_t)ns + 1);
    int64_t sum = 0;
    for (int64_t i = a; i < b; ++i) sum += off[i];
    sh[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? sh[t - 1] : 0;
    for (int64_t i = a; i < b; ++i) {
        run += off[i];
        off[i] = run;
    }
}

// Step 2b (after the scan; only when the copy fits its cap): base[off[c] / 256 + k] = the
// smallest col - row at position k over the rows of slice c that have one (0 if none);
// sets *over when a residual would exceed 16 bits.
__global__ void __launch_bounds__(256) slice_base_kernel(int n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const int64_t* __restrict__ off, int64_t cap,
                                                         int32_t* __restrict__ base,
                                                         unsigned long long* __restrict__ over) {
    __shared__ int smin[4], smax[4];
    const int ns = gridDim.x;
    if (off[ns] > cap) return;        // the copy is not built
    const int c = blockIdx.x, t = threadIdx.x, row = c * 256 + t;
    const int64_t b0 = off[c];
    const int w = (int)((off[c + 1] - b0) / 256);
    int a = 0, len = 0;
    if (row < n) { a = rp[row]; len = rp[row + 1] - a; }
    bool bad = false;
    for (int k = 0; k < w; ++k) {
        int lo = INT_MAX, hi = INT_MIN;
        if (k < len) lo = hi = ci[a + k] - row;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o));
            hi = max(hi, __shfl_xor(hi, o));
        }
        if ((t & 63) == 0) { smin[t >> 6] = lo; smax[t >> 6] = hi; }
        __syncthreads();
        lo = min(min(smin[0], smin[1]), min(smin[2], smin[3]));
        hi = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
        __syncthreads();
        if (t == 0) base[b0 / 256 + k] = lo == INT_MAX ? 0 : lo;
        if (lo != INT_MAX && (int64_t)hi - (int64_t)lo > 65535) bad = true;
    }
    if (t == 0 && bad) atomicOr(over, 1ull);
}

// Step 3: copy every row into its slice (lane t of block c: row 256c + t); D16: the column
// entries as 16-bit residuals col - row - base[c][k] (the caller checked that all fit).
template <class VT, bool D16>
__global__ void __launch_bounds__(256) slice_fill_kernel(int n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const VT* __restrict__ val,
                                                         const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ sbase,
                                                         int32_t* __restrict__ scol, VT* __restrict__ sval) {
    const int c = blockIdx.x, t = threadIdx.x, row = c * 256 + t;
    const int64_t base = off[c];
    const int w = (int)((off[c + 1] - base) / 256);
    int a = 0, len = 0;
    if (row < n) { a = rp[row]; len = rp[row + 1] - a; }
    uint16_t* dcol = (uint16_t*)scol;
    for (int k = 0; k < w; ++k) {
        const int64_t i = base + (int64_t)k * 256 + t;
        if constexpr (D16)
            dcol[i] = k < len ? (uint16_t)(ci[a + k] - row - sbase[base / 256 + k]) : (uint16_t)0;
        else
            scol[i] = k < len ? ci[a + k] : 0;
        sval[i] = k < len ? val[a + k] : VT(0);
    }
}

// Offset form, step 1 (one block per slice): the slice's distinct offsets col - row in
// ascending order into ofs[c][0 .. K) (unused slots 0), and off[c + 1] = 256 K; a slice with
// more than OFS_MAX offsets sets *over.  Each round finds the smallest offset above the
// previous one over the whole slice (lane minima, wave shuffles, then the 4 waves).
__global__ void __launch_bounds__(256) ofs_scan_kernel(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, int64_t* __restrict__ off,
                                                       int32_t* __restrict__ ofs, int* __restrict__ over) {
    __shared__ long long smin[4];
    const int c = blockIdx.x, t = threadIdx.x, row = c * 256 + t;
    int a = 0, e = 0;
    if (row < n) { a = rp[row]; e = rp[row + 1]; }
    long long last = LLONG_MIN;
    int K = 0;
    for (int j = 0; j <= OFS_MAX; ++j) {
        long long lo = LLONG_MAX;   // smallest offset of the row above `last` (columns ascend)
        for (int k = a; k < e; ++k) {
            const long long d = (long long)ci[k] - row;
            if (d > last) { lo = d; break; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lo = min(lo, (long long)__shfl_xor(lo, o));
        if ((t & 63) == 0) smin[t >> 6] = lo;
        __syncthreads();
        lo = min(min(smin[0], smin[1]), min(smin[2], smin[3]));
        __syncthreads();
        if (lo == LLONG_MAX) break;           // uniform over the block
        if (j == OFS_MAX) {                   // one offset too many
            if (t == 0) atomicOr(over, 1);
            break;
        }
        if (t == 0) ofs[(int64_t)c * OFS_MAX + j] = (int32_t)lo;
        last = lo;
        K = j + 1;
    }
    if (t < OFS_MAX && t >= K) ofs[(int64_t)c * OFS_MAX + t] = 0;
    if (t == 0) {
        off[c + 1] = 256LL * K;
        if (c == 0) off[0] = 0;
    }
}

// Offset form, step 2 (one block per slice, after the prefix sums of off): slot values and
// mask bytes of every row (rows past n: mask 0, values 0).
template <class VT>
__global__ void __launch_bounds__(256) ofs_fill_kernel(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const VT* __restrict__ val,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ ofs, uint8_t* __restrict__ mask,
                                                       VT* __restrict__ sval) {
    const int c = blockIdx.x, t = threadIdx.x, row = c * 256 + t;
    const int64_t base = off[c];
    const int K = (int)((off[c + 1] - base) / 256);
    int a = 0, e = 0;
    if (row < n) { a = rp[row]; e = rp[row + 1]; }
    uint32_t m = 0;
    int k = a;
    for (int j = 0; j < K; ++j) {
        const long long d = ofs[(int64_t)c * OFS_MAX + j];
        VT v = VT(0);
        if (k < e && (long long)ci[k] - row == d) {
            v = val[k];
            m |= 1u << j;
            ++k;
        }
        sval[base + (int64_t)j * 256 + t] = v;
    }
    mask[row] = (uint8_t)m;
}

// Row-sorted copy, step 1: perm over each window of WSORT rows, by decreasing row length
// (ties: ascending row), one block of 1024 threads per window (bitonic sort in LDS of the
// keys (INT_MAX - len) << 32 | local row, which are distinct).
__global__ void __launch_bounds__(1024) wslice_sort_kernel(int n, const int32_t* __restrict__ rp,
                                                           int32_t* __restrict__ perm) {
    __shared__ unsigned long long key[WSORT];
    const int r0 = blockIdx.x * WSORT;
    for (int j = threadIdx.x; j < WSORT; j += blockDim.x) {
        const int r = r0 + j;
        key[j] = r < n ? ((unsigned long long)(uint32_t)(0x7fffffff - (rp[r + 1] - rp[r])) << 32) | (uint32_t)j
                       : ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= WSORT; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < WSORT; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = key[i], b = key[l];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < WSORT; j += blockDim.x) {
        const int r = r0 + j;
        if (r < n) perm[r] = r0 + (int)(uint32_t)(key[j] & 0xffffffffull);
    }
}

// Step 2: off[c + 1] = 64 * (longest row of wave slice c), off[0] = 0 (blocks of 256 = 4
// slices; nws slices in all).
__global__ void __launch_bounds__(256) wslice_width_kernel(int n, int nws, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ perm,
                                                           int64_t* __restrict__ off) {
    const int slot = blockIdx.x * 256 + threadIdx.x;
    const int ws = slot / WS_ROWS;
    int len = 0;
    if (slot < n) {
        const int r = perm[slot];
        len = rp[r + 1] - rp[r];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o));
    if ((threadIdx.x & 63) == 0 && ws < nws) off[ws + 1] = (int64_t)WS_ROWS * len;
    if (slot == 0) off[0] = 0;
}

// Step 3 (after the scan): copy every row into its slot, column-major per wave slice.
template <class VT>
__global__ void __launch_bounds__(256) wslice_fill_kernel(int n, int nws, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const VT* __restrict__ val,
                                                          const int32_t* __restrict__ perm,
                                                          const int64_t* __restrict__ off,
                                                          int32_t* __restrict__ scol, VT* __restrict__ sval) {
    const int slot = blockIdx.x * 256 + threadIdx.x;
    const int ws = slot / WS_ROWS, lane = slot % WS_ROWS;
    if (ws >= nws) return;
    const int64_t base = off[ws];
    const int w = (int)((off[ws + 1] - base) / WS_ROWS);
    int a = 0, len = 0;
    if (slot < n) {
        const int r = perm[slot];
        a = rp[r];
        len = rp[r + 1] - a;
    }
    for (int k = 0; k < w; ++k) {
        const int64_t i = base + (int64_t)k * WS_ROWS + lane;
        scol[i] = k < len ? ci[a + k] : 0;
        sval[i] = k < len ? val[a + k] : VT(0);
    }
}

// ----------------------------------------------------------------------------- dot sites
#define XD_SHARED(D)                                   \
    __shared__ unsigned long long sh_acc[(D) * xd::NCH]; \
    __shared__ long long sh_tmp[(D) * xd::NCH];          \
    __shared__ uint32_t sh_flags[(D)];                   \
    __shared__ int sh_rng[2 * (D)];

// Exact element-wise fused kernel.  Op provides:
//   load()                      read device scalars
//   ld(i, in[NIN])              global loads of element i
//   st(i, in, xa[D], ya[D])     updates and stores of element i; dot operands
//   finalize(const double* d)   run by a finalize role (XFin) once the records are summed
// U elements per lane and trip: all U elements' loads are issued before the dependent
// exact-accumulation work of the first (the result is the exact sum whatever the order).
// QUEUE (single dots): products outside TwoProd's range go through each wave's LDS queue
// and are deposited 64 at a time (xd::accumulate_q) instead of by the few lanes that meet
// them while the rest of the wave waits.
template <int D, int K, class Op, int U = 2, bool QUEUE = false>
__global__ void __launch_bounds__(1024)
ew_dot_kernel(Op op, int64_t n, xd::Site site, const int* halt, int* seen) {
    if (halt && *halt) {
        if (seen && blockIdx.x == 0 && threadIdx.x == 0) *seen = 1;
        return;
    }
    XD_SHARED(D)
    constexpr int QW = QUEUE ? 16 : 1;
    __shared__ double sh_qx[QW][128], sh_qy[QW][128];
    __shared__ int sh_qn[QW];
    double* qx = sh_qx[QUEUE ? (threadIdx.x >> 6) : 0];
    double* qy = sh_qy[QUEUE ? (threadIdx.x >> 6) : 0];
    int* qn = &sh_qn[QUEUE ? (threadIdx.x >> 6) : 0];
    if (QUEUE && (threadIdx.x & 63) == 0) *qn = 0;
    xd::block_init<D>(sh_acc, sh_flags);
    op.load();
    double e[D][K];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k = 0; k < K; ++k) e[d][k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        double in[U][Op::NIN];
#pragma unroll
        for (int u = 0; u < U; ++u) op.ld(i + u * stride, in[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double xa[D], ya[D];
            op.st(i + u * stride, in[u], xa, ya);
#pragma unroll
            for (int d = 0; d < D; ++d)
                if constexpr (QUEUE) xd::accumulate_q<K>(e[d], xa[d], ya[d], sh_acc, &sh_flags[d], qx, qy, qn);
                else xd::accumulate<K>(e[d], xa[d], ya[d], sh_acc + d * xd::NCH, &sh_flags[d]);
        }
    }
    for (; i < n; i += stride) {
        double in[Op::NIN];
        op.ld(i, in);
        double xa[D], ya[D];
        op.st(i, in, xa, ya);
#pragma unroll
        for (int d = 0; d < D; ++d)
            if constexpr (QUEUE) xd::accumulate_q<K>(e[d], xa[d], ya[d], sh_acc, &sh_flags[d], qx, qy, qn);
            else xd::accumulate<K>(e[d], xa[d], ya[d], sh_acc + d * xd::NCH, &sh_flags[d]);
    }
    if constexpr (QUEUE) xd::drain_queue(sh_acc, qx, qy, qn);
    xd::block_flush<D, K>(e, sh_acc);
    xd::block_write<D>(site, sh_acc, sh_flags, sh_tmp, sh_rng);
}

// Exact SpMV with an epilogue that returns D dot operands for its row.
// Epi: load(); row(int row, double s, double xa[D], double ya[D]); finalize(const double*)
template <int L, int D, int K, class VT, class Epi>
__global__ void __launch_bounds__(256)
spmv_dot_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                const VT* __restrict__ val, const double* __restrict__ x, Epi epi,
                xd::Site site, const int* halt) {
    if (halt && *halt) return;
    XD_SHARED(D)
    xd::block_init<D>(sh_acc, sh_flags);
    epi.load();
    double e[D][K];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k = 0; k < K; ++k) e[d][k] = 0.0;
    const int groups = blockDim.x / L;
    const int lane = threadIdx.x % L;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int stride = gridDim.x * groups;
    for (int row = blk * groups + (int)threadIdx.x / L; row < n; row += stride) {
        const int a = rp[row], b = rp[row + 1];
        double s = 0.0;
        for (int k = a + lane; k < b; k += L) {
            double prod = (double)val[k] * x[ci[k]];
            s = s + prod;
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) s = s + __shfl_xor(s, o);
        if (lane == 0) {
            double xa[D], ya[D];
            epi.row(row, s, xa, ya);
#pragma unroll
            for (int d = 0; d < D; ++d)
                xd::accumulate<K>(e[d], xa[d], ya[d], sh_acc + d * xd::NCH, &sh_flags[d]);
        }
    }
    xd::block_flush<D, K>(e, sh_acc);
    xd::block_write<D>(site, sh_acc, sh_flags, sh_tmp, sh_rng);
}

// Row-sequential SpMV with D exact dots in the epilogue (persistent grid).
template <int D, int K, class Epi>
struct DotBody {
    Epi& epi;
    double (&e)[D][K];
    unsigned long long* acc;
    uint32_t* flags;
    __device__ __forceinline__ void operator()(int row, double s) {
        double xa[D], ya[D];
        epi.row(row, s, xa, ya);
#pragma unroll
        for (int d = 0; d < D; ++d) xd::accumulate<K>(e[d], xa[d], ya[d], acc + d * xd::NCH, &flags[d]);
    }
};

template <int D, int K, class VT, class Epi, bool SL = false, int SLF = 0>
__global__ void __launch_bounds__(256)
spmv_seq_dot_kernel(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                    const VT* __restrict__ val, const double* __restrict__ x, Epi epi,
                    xd::Site site, const int* halt, Sliced<VT> sl) {
    if (halt && *halt) return;
    XD_SHARED(D)
    __shared__ double sprod[SL ? 2 : SEQ_CAP];
    xd::block_init<D>(sh_acc, sh_flags);
    epi.load();
    double e[D][K];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k = 0; k < K; ++k) e[d][k] = 0.0;
    DotBody<D, K, Epi> body{epi, e, sh_acc, sh_flags};
    seq_stage<SEQ_CAP, VT, double, double, DotBody<D, K, Epi>, false, SL, SLF>(n, rp, ci, val, x, 0,
                                                                                 (int)gridDim.x, sprod, body, sl);
    xd::block_flush<D, K>(e, sh_acc);
    xd::block_write<D>(site, sh_acc, sh_flags, sh_tmp, sh_rng);
}

// ----------------------------------------------------------------------------- FP32 plain dots

// Plain FP32 dots: per-thread sequential sums in grid-stride order, xor-butterfly
// within the wave, waves in index order; the per-block partials are summed in a fixed
// tree by a finalize role (FFin; deterministic for a given launch shape).
// An op with SPLIT provides ld(i, in[NIN]) and st(i, in, xa, ya): the kernel then issues
// the loads of two elements before computing either (more loads in flight per lane).
template <class Op, class = void>
struct fsplit : std::false_type {};
template <class Op>
struct fsplit<Op, std::void_t<decltype(Op::SPLIT)>> : std::bool_constant<Op::SPLIT> {};

template <class T, int D, class Op>
__global__ void __launch_bounds__(1024)
ew_fdot_kernel(Op op, int64_t n, TSite<T> site, const int* halt, int* seen) {
    if (halt && *halt) {
        if (seen && blockIdx.x == 0 && threadIdx.x == 0) *seen = 1;
        return;
    }
    __shared__ T sh_w[D][16];
    op.load();
    T a[D];
#pragma unroll
    for (int d = 0; d < D; ++d) a[d] = T(0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if constexpr (fsplit<Op>::value) {
        // elements i and i + stride per trip, accumulated in that order (the same sums as
        // one element per trip)
        int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        for (; i + stride < n; i += 2 * stride) {
            T ia[Op::NIN], ib[Op::NIN];
            op.ld(i, ia);
            op.ld(i + stride, ib);
            T xa[D], ya[D];
            op.st(i, ia, xa, ya);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                T p = xa[d] * ya[d];
                a[d] = a[d] + p;
            }
            op.st(i + stride, ib, xa, ya);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                T p = xa[d] * ya[d];
                a[d] = a[d] + p;
            }
        }
        if (i < n) {
            T ia[Op::NIN];
            op.ld(i, ia);
            T xa[D], ya[D];
            op.st(i, ia, xa, ya);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                T p = xa[d] * ya[d];
                a[d] = a[d] + p;
            }
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            T xa[D], ya[D];
            op.elem(i, xa, ya);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                T p = xa[d] * ya[d];
                a[d] = a[d] + p;
            }
        }
    }
    const int wid = threadIdx.x / xd::WAVE, nw = blockDim.x / xd::WAVE;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        T v = a[d];
#pragma unroll
        for (int o = xd::WAVE / 2; o > 0; o >>= 1) v = v + __shfl_xor(v, o);
        if ((threadIdx.x & (xd::WAVE - 1)) == 0) sh_w[d][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < D) {
        T s = T(0);
        for (int w = 0; w < nw; ++w) s = s + sh_w[threadIdx.x][w];
        site.part[(size_t)blockIdx.x * D + threadIdx.x] = s;
    }
}

// Element interface (elem(i, xa, ya)) over an exact-dot op (ld / st), so that an FP64
// phase can run with plain tree dots.
template <class Op>
struct ElemOf {
    Op op;
    __device__ __forceinline__ void load() { op.load(); }
    __device__ __forceinline__ void elem(int64_t i, double (&xa)[Op::ND], double (&ya)[Op::ND]) {
        double in[Op::NIN];
        op.ld(i, in);
        op.st(i, in, xa, ya);
    }
    __device__ __forceinline__ void finalize(const double* d) { op.finalize(d); }
};

// ----------------------------------------------------------------------------- small kernels
template <class F>
__global__ void __launch_bounds__(256) ew_kernel(F f, int64_t n, const int* halt) {
    if (halt && *halt) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) f(i);
}

template <class F>
__global__ void single_kernel(F f) {
    if (threadIdx.x == 0 && blockIdx.x == 0) f();
}

// ============================================================================= p-BiCGStab ops
// Loads and stores of the phases' vectors.  NT: non-temporal (streamed past the caches),
// chosen when the iteration's working set exceeds the Infinity Cache: the vectors then
// do not evict the matrix, which both SpMVs of the iteration read whole.  The operand of
// the SpMV that follows a phase (z, w) keeps plain stores: that SpMV gathers it next.
template <bool NT, class T>
__device__ __forceinline__ T get(const T* p, int64_t i) {
    if constexpr (NT) return __builtin_nontemporal_load(p + i);
    else return p[i];
}

template <bool NT, class T>
__device__ __forceinline__ void put(T* p, int64_t i, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p + i);
    else p[i] = v;
}

// Phase A (Algorithm 2, the p, s, z, q, y updates) + (q,y), (y,y), (r_hat,s), (r_hat,z).
template <class Fin, bool NT = false>
struct PhaseA {
    const double* r; const double* w; const double* t; const double* v; const double* rhat;
    double* p; double* s; double* z; double* q; double* y;
    const double* scal;  // alpha, beta, omega
    int first;
    Fin fin;
    double alpha, beta, omega;
    static constexpr int ND = 4;
    static constexpr int NIN = 8;
    __device__ __forceinline__ void load() { alpha = scal[0]; beta = scal[1]; omega = scal[2]; }
    __device__ __forceinline__ void ld(int64_t i, double (&in)[NIN]) const {
        in[0] = get<NT>(r, i); in[1] = get<NT>(w, i); in[2] = get<NT>(t, i); in[3] = get<NT>(rhat, i);
        if (!first) {
            in[4] = get<NT, double>(p, i); in[5] = get<NT, double>(s, i);
            in[6] = get<NT, double>(z, i); in[7] = get<NT>(v, i);
        }
    }
    __device__ __forceinline__ void st(int64_t i, const double (&in)[NIN], double (&xa)[4], double (&ya)[4]) {
        const double ri = in[0], wi = in[1], ti = in[2];
        double pi, si, zi;
        if (first) {
            pi = ri; si = wi; zi = ti;
        } else {
            pi = ri + beta * (in[4] - omega * in[5]);
            si = wi + beta * (in[5] - omega * in[6]);
            zi = ti + beta * (in[6] - omega * in[7]);
        }
        const double qi = ri - alpha * si;
        const double yi = wi - alpha * zi;
        put<NT>(p, i, pi); put<NT>(s, i, si); put<false>(z, i, zi); put<NT>(q, i, qi); put<NT>(y, i, yi);
        const double rh = in[3];
        xa[0] = qi; ya[0] = yi;
        xa[1] = yi; ya[1] = yi;
        xa[2] = rh; ya[2] = si;
        xa[3] = rh; ya[3] = zi;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// Phase B (x, r, w updates) + (r_hat,r), (r_hat,w), (r,r).
template <class Fin, bool NT = false>
struct PhaseB {
    double* x; const double* p; const double* q; const double* y; const double* t; const double* v;
    const double* rhat; double* r; double* w;
    const double* scal;
    Fin fin;
    double alpha, omega;
    static constexpr int ND = 3;
    static constexpr int NIN = 7;
    __device__ __forceinline__ void load() { alpha = scal[0]; omega = scal[2]; }
    __device__ __forceinline__ void ld(int64_t i, double (&in)[NIN]) const {
        in[0] = get<NT, double>(x, i); in[1] = get<NT>(p, i); in[2] = get<NT>(q, i); in[3] = get<NT>(y, i);
        in[4] = get<NT>(t, i); in[5] = get<NT>(v, i); in[6] = get<NT>(rhat, i);
    }
    __device__ __forceinline__ void st(int64_t i, const double (&in)[NIN], double (&xa)[3], double (&ya)[3]) {
        const double qi = in[2], yi = in[3];
        const double xi = (in[0] + alpha * in[1]) + omega * qi;
        const double ri = qi - omega * yi;
        const double wi = yi - omega * (in[4] - alpha * in[5]);
        put<NT>(x, i, xi); put<NT>(r, i, ri); put<false>(w, i, wi);
        const double rh = in[6];
        xa[0] = rh; ya[0] = ri;
        xa[1] = rh; ya[1] = wi;
        xa[2] = ri; ya[2] = ri;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// Plain dots of given vectors (D <= 4); no updates.  NT: the vectors are read with
// non-temporal loads (a standalone dot over vectors larger than the Infinity Cache).
template <int D, class Fin, bool NT = false>
struct DotsOp {
    const double* a[4];
    const double* b[4];
    Fin fin;
    static constexpr int ND = D;
    static constexpr int NIN = 2 * D;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void ld(int64_t i, double (&in)[NIN]) const {
#pragma unroll
        for (int d = 0; d < D; ++d) { in[2 * d] = get<NT>(a[d], i); in[2 * d + 1] = get<NT>(b[d], i); }
    }
    __device__ __forceinline__ void st(int64_t, const double (&in)[NIN], double (&xa)[D], double (&ya)[D]) const {
#pragma unroll
        for (int d = 0; d < D; ++d) { xa[d] = in[2 * d]; ya[d] = in[2 * d + 1]; }
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// finalizers ----------------------------------------------------------------
struct FinStore {            // write the D results to out[]
    double* out;
    int D;
    __device__ void operator()(const double* d) const {
        for (int k = 0; k < D; ++k) out[k] = d[k];
    }
};

struct FinStoreF {           // one FP32 result to out[0]
    float* out;
    __device__ void operator()(const float* d) const { out[0] = d[0]; }
};

__device__ __forceinline__ bool fin3(double a, double b, double c) { return isfinite(a) && isfinite(b) && isfinite(c); }

// ||b||^2 -> normb
struct FinNormB {
    State* st;
    __device__ void operator()(const double* d) const {
        double nb2 = d[0];
        if (!isfinite(nb2)) {
            st->normb = __longlong_as_double(0x7ff8000000000000ll);
            st->halt = 1; st->reason |= R_NONFINITE; return;
        }
        double nb = sqrt(nb2);
        st->normb = nb;
        if (nb == 0.0) { st->halt = 1; st->reason |= R_ZERO_RHS; }
    }
};

// The stopping test: the first true-residual test comes when rec <= tol; after a
// failed test (check_it = its iteration) the next comes 5 iterations later.
__device__ __forceinline__ bool true_test_due(const State* st, double rec, int it) {
    if (st->check_it < 0) return rec <= st->tol;
    return it - st->check_it >= 5;
}

// initial (r_hat, r0), (r_hat, w0), (r0, r0) -> rho, alpha0, rec
struct FinInitP {
    State* st;
    __device__ void operator()(const double* d) const {
        double rho = d[0], rw = d[1], rr = d[2];
        double rec = sqrt(rr) / st->normb;
        st->rec = rec; st->rho = rho; st->rw = rw;
        int reason = 0;
        if (true_test_due(st, rec, 0)) reason |= R_CHECK;
        if (!isfinite(rho) || !isfinite(rw)) reason |= R_NONFINITE;
        else if (rw == 0.0) reason |= R_BREAKDOWN;
        else st->alpha = rho / rw;
        st->beta = 0.0; st->omega = 0.0;
        if (reason) { st->halt = 1; st->reason |= reason; }
    }
};

// after phase A / after y = A q: omega = (q,y)/(y,y) (+ store (r_hat,s), (r_hat,z))
struct FinOmega {
    State* st;
    int has_rsz;
    __device__ void operator()(const double* d) const {
        double qy = d[0], yy = d[1];
        st->qy = qy; st->yy = yy;
        bool fin = isfinite(qy) && isfinite(yy);
        if (has_rsz) {
            st->rs = d[2]; st->rz = d[3];
            fin = fin && isfinite(d[2]) && isfinite(d[3]);
        }
        if (!fin) { st->halt = 1; st->reason |= R_NONFINITE; return; }
        if (yy == 0.0) { st->halt = 1; st->reason |= R_YYZERO; return; }
        double om = qy / yy;
        st->omega = om;
        if (om == 0.0) { st->halt = 1; st->reason |= R_BREAKDOWN; }
    }
};

// after phase B: rho', beta, alpha', rec, iteration count, halts
struct FinPhaseB {
    State* st;
    __device__ void operator()(const double* d) const {
        const double rho_new = d[0], rw = d[1], rr = d[2];
        const double alpha = st->alpha, omega = st->omega, rho = st->rho;
        const int it = st->iter + 1;
        st->iter = it;
        const double rec = sqrt(rr) / st->normb;
        st->rec = rec; st->rw = rw; st->rr = rr;
        if (st->hist && it <= st->hist_len) st->hist[it - 1] = rec;
        bool stall = false;
        if (st->stall_hist) {
            st->stall_hist[it - 1] = rec;
            const int W = st->stall_window;
            stall = W > 0 && it > W && rec > 0.5 * st->stall_hist[it - 1 - W];
        }
        const double beta = ((alpha / omega) * rho_new) / rho;
        const double den = (rw + beta * st->rs) - (beta * omega) * st->rz;
        const double alpha_new = den != 0.0 ? rho_new / den : __longlong_as_double(0x7ff8000000000000ll);
        int reason = 0;
        if (true_test_due(st, rec, it)) reason |= R_CHECK;
        bool nonfin = !(isfinite(rho_new) && isfinite(rw) && isfinite(rr) && isfinite(beta)) ||
                      (den != 0.0 && !isfinite(alpha_new));
        if (nonfin) reason |= R_NONFINITE;
        else if (rho_new == 0.0 || den == 0.0) reason |= R_BREAKDOWN;
        else { st->beta = beta; st->alpha = alpha_new; st->rho = rho_new; }
        if (stall) reason |= R_STALL;
        if (it >= st->max_iter) reason |= R_MAXIT;
        if (reason) { st->halt = 1; st->reason |= reason; }
    }
};

// BiCGStab initial (r_hat, r0), (r0, r0) -> rho, rec
struct FinInitB {
    State* st;
    __device__ void operator()(const double* d) const {
        double rho = d[0], rr = d[1];
        double rec = sqrt(rr) / st->normb;
        st->rec = rec; st->rho = rho;
        st->alpha = 0.0; st->beta = 0.0; st->omega = 0.0;
        int reason = 0;
        if (true_test_due(st, rec, 0)) reason |= R_CHECK;
        if (!isfinite(rho)) reason |= R_NONFINITE;
        if (reason) { st->halt = 1; st->reason |= reason; }
    }
};

// refinement: nu = sqrt((r,r)), rel = nu / ||b||
struct FinIR {
    State* st;
    __device__ void operator()(const double* d) const {
        double nu = sqrt(d[0]);
        st->last_dot = nu;
        st->true_rel = nu / st->normb;
    }
};

// true residual: (res,res) -> true_rel
struct FinTrue {
    State* st;
    int count;   // 1: a stopping test (counted in true_checks); 0: the final report
    __device__ void operator()(const double* d) const {
        st->true_rel = sqrt(d[0]) / st->normb;
        st->true_checks += count;
    }
};

// true residual for the history: out = sqrt((res,res)) / ||b||, the state untouched
struct FinTrueHist {
    const State* st;
    double* out;
    __device__ void operator()(const double* d) const { *out = sqrt(d[0]) / st->normb; }
};

// epilogue for res = b - A x with the dot (res,res)
template <class Fin>
struct EpiResidDot {
    const double* b;
    double* res;
    Fin fin;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void row(int i, double s, double (&xa)[1], double (&ya)[1]) {
        double v = b[i] - s;
        res[i] = v;
        xa[0] = v; ya[0] = v;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// ============================================================================= BiCGStab ops
// s = A p with (r_hat, s) -> alpha = rho / (r_hat, s)
struct FinAlphaB {
    State* st;
    __device__ void operator()(const double* d) const {
        double rs = d[0];
        st->rs = rs;
        if (!isfinite(rs)) { st->halt = 1; st->reason |= R_NONFINITE; return; }
        if (rs == 0.0 || st->rho == 0.0) { st->halt = 1; st->reason |= R_BREAKDOWN; return; }
        st->alpha = st->rho / rs;
    }
};

template <bool NT = false>
struct EpiSDot {
    double* s; const double* rhat; FinAlphaB fin;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void row(int i, double v, double (&xa)[1], double (&ya)[1]) {
        put<NT>(s, i, v); xa[0] = get<NT>(rhat, i); ya[0] = v;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// y = A q with (q,y), (y,y)
template <bool NT = false>
struct EpiYDot {
    double* y; const double* q; FinOmega fin;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void row(int i, double v, double (&xa)[2], double (&ya)[2]) {
        put<NT>(y, i, v);
        double qi = get<NT>(q, i);
        xa[0] = qi; ya[0] = v;
        xa[1] = v; ya[1] = v;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// x = (x + alpha p) + omega q; r = q - omega y; (r_hat, r), (r, r)
struct FinBiCGStabXR {
    State* st;
    __device__ void operator()(const double* d) const {
        const double rho_new = d[0], rr = d[1];
        const double alpha = st->alpha, omega = st->omega, rho = st->rho;
        const int it = st->iter + 1;
        st->iter = it;
        const double rec = sqrt(rr) / st->normb;
        st->rec = rec; st->rr = rr;
        if (st->hist && it <= st->hist_len) st->hist[it - 1] = rec;
        const double beta = ((alpha / omega) * rho_new) / rho;
        int reason = 0;
        if (true_test_due(st, rec, it)) reason |= R_CHECK;
        if (!(isfinite(rho_new) && isfinite(rr) && isfinite(beta))) reason |= R_NONFINITE;
        else if (rho_new == 0.0) reason |= R_BREAKDOWN;
        else { st->beta = beta; st->rho = rho_new; }
        if (it >= st->max_iter) reason |= R_MAXIT;
        if (reason) { st->halt = 1; st->reason |= reason; }
    }
};

template <bool NT = false>
struct OpBiCGStabXR {
    double* x; const double* p; const double* q; const double* y; const double* rhat; double* r;
    const double* scal; FinBiCGStabXR fin;
    double alpha, omega;
    static constexpr int NIN = 5;
    __device__ __forceinline__ void load() { alpha = scal[0]; omega = scal[2]; }
    __device__ __forceinline__ void ld(int64_t i, double (&in)[NIN]) const {
        in[0] = get<NT, double>(x, i); in[1] = get<NT>(p, i); in[2] = get<NT>(q, i); in[3] = get<NT>(y, i);
        in[4] = get<NT>(rhat, i);
    }
    __device__ __forceinline__ void st(int64_t i, const double (&in)[NIN], double (&xa)[2], double (&ya)[2]) {
        const double qi = in[2];
        const double xi = (in[0] + alpha * in[1]) + omega * qi;
        const double ri = qi - omega * in[3];
        put<NT>(x, i, xi); put<NT>(r, i, ri);
        xa[0] = in[4]; ya[0] = ri;
        xa[1] = ri; ya[1] = ri;
    }
    __device__ __forceinline__ void finalize(const double* d) { fin(d); }
};

// ============================================================================= FP32 inner solver ops
template <class Fin, bool NT = false>
struct FPhaseA {
    const float* r; const float* w; const float* t; const float* v; const float* rhat;
    float* p; float* s; float* z; float* q; float* y;
    const float* scal; int first; Fin fin;
    float alpha, beta, omega;
    static constexpr bool SPLIT = true;
    static constexpr int NIN = 8;
    __device__ __forceinline__ void load() { alpha = scal[0]; beta = scal[1]; omega = scal[2]; }
    __device__ __forceinline__ void ld(int64_t i, float (&in)[NIN]) const {
        in[0] = get<NT>(r, i); in[1] = get<NT>(w, i); in[2] = get<NT>(t, i); in[3] = get<NT>(rhat, i);
        if (!first) {
            in[4] = get<NT, float>(p, i); in[5] = get<NT, float>(s, i);
            in[6] = get<NT, float>(z, i); in[7] = get<NT>(v, i);
        }
    }
    __device__ __forceinline__ void st(int64_t i, const float (&in)[NIN], float (&xa)[4], float (&ya)[4]) {
        const float ri = in[0], wi = in[1], ti = in[2];
        float pi, si, zi;
        if (first) { pi = ri; si = wi; zi = ti; }
        else {
            const float pp = in[4], sp = in[5], zp = in[6], vp = in[7];
            pi = ri + beta * (pp - omega * sp);
            si = wi + beta * (sp - omega * zp);
            zi = ti + beta * (zp - omega * vp);
        }
        const float qi = ri - alpha * si;
        const float yi = wi - alpha * zi;
        put<NT>(p, i, pi); put<NT>(s, i, si); put<false>(z, i, zi); put<NT>(q, i, qi); put<NT>(y, i, yi);
        const float rh = in[3];
        xa[0] = qi; ya[0] = yi;
        xa[1] = yi; ya[1] = yi;
        xa[2] = rh; ya[2] = si;
        xa[3] = rh; ya[3] = zi;
    }
    __device__ __forceinline__ void finalize(const float* d) { fin(d); }
};

template <class Fin, bool NT = false>
struct FPhaseB {
    float* x; const float* p; const float* q; const float* y; const float* t; const float* v;
    const float* rhat; float* r; float* w; const float* scal; Fin fin;
    float alpha, omega;
    static constexpr bool SPLIT = true;
    static constexpr int NIN = 7;
    __device__ __forceinline__ void load() { alpha = scal[0]; omega = scal[2]; }
    __device__ __forceinline__ void ld(int64_t i, float (&in)[NIN]) const {
        in[0] = get<NT>(q, i); in[1] = get<NT>(y, i); in[2] = get<NT, float>(x, i); in[3] = get<NT>(p, i);
        in[4] = get<NT>(t, i); in[5] = get<NT>(v, i); in[6] = get<NT>(rhat, i);
    }
    __device__ __forceinline__ void st(int64_t i, const float (&in)[NIN], float (&xa)[3], float (&ya)[3]) {
        const float qi = in[0], yi = in[1];
        const float xi = (in[2] + alpha * in[3]) + omega * qi;
        const float ri = qi - omega * yi;
        const float wi = yi - omega * (in[4] - alpha * in[5]);
        put<NT>(x, i, xi); put<NT>(r, i, ri); put<false>(w, i, wi);
        const float rh = in[6];
        xa[0] = rh; ya[0] = ri;
        xa[1] = rh; ya[1] = wi;
        xa[2] = ri; ya[2] = ri;
    }
    __device__ __forceinline__ void finalize(const float* d) { fin(d); }
};

template <int D, class Fin>
struct FDotsOp {
    const float* a[4]; const float* b[4]; Fin fin;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void elem(int64_t i, float (&xa)[D], float (&ya)[D]) {
#pragma unroll
        for (int d = 0; d < D; ++d) { xa[d] = a[d][i]; ya[d] = b[d][i]; }
    }
    __device__ __forceinline__ void finalize(const float* d) { fin(d); }
};

// (b,b), (r_hat,r), (r_hat,w) of the inner solve (r = r_hat = b at x0 = 0)
// Restart of the FP32 process (r_hat = r, p = r, s = w, z = t follow in phase A):
// d = (r_hat, r), (r_hat, w) -> rho, alpha = rho / (r_hat, w); beta = omega = 0.
struct FFinRestart {
    FState* st;
    __device__ void operator()(const float* d) const {
        const float rho = d[0], rw = d[1];
        st->beta = 0.0f; st->omega = 0.0f;
        if (rw == 0.0f || !isfinite(rw)) { st->halt = 1; st->reason |= R_BREAKDOWN; return; }
        st->rho = rho;
        st->alpha = rho / rw;
    }
};

// Continuation after a reliable update (r, w, t, s, z, v rebuilt; beta, omega kept):
// d = (r_hat, r), (r_hat, w), (r_hat, s), (r_hat, z);
// alpha = rho / (((r_hat, w) + beta (r_hat, s)) - (beta omega)(r_hat, z)).
struct FFinReplace {
    FState* st;
    __device__ void operator()(const float* d) const {
        const float rho = d[0];
        const float beta = st->beta, omega = st->omega;
        const float den = (d[1] + beta * d[2]) - (beta * omega) * d[3];
        if (rho == 0.0f || den == 0.0f || !isfinite(den)) { st->halt = 1; st->reason |= R_BREAKDOWN; return; }
        st->rho = rho;
        st->alpha = rho / den;
    }
};

struct FFinOmega {
    FState* st;
    __device__ void operator()(const float* d) const {
        float qy = d[0], yy = d[1];
        st->rs = d[2]; st->rz = d[3];
        if (yy == 0.0f || !isfinite(yy)) { st->halt = 1; st->reason |= (yy == 0.0f ? R_YYZERO : R_NONFINITE); return; }
        float om = qy / yy;
        if (om == 0.0f || !isfinite(om)) { st->halt = 1; st->reason |= R_BREAKDOWN; return; }
        st->omega = om;
    }
};

// End of an FP32 iteration: beta, alpha for the next one, then the stop reasons of the
// refinement (R_CONVERGED: rec <= lim; R_CHECK: rec <= tol, a reliable update is due;
// R_BREAKDOWN; R_STALL: no new minimum of rec for `stall` iterations; R_MAXIT).
struct FFinRU {
    FState* st;
    __device__ void operator()(const float* d) const {
        const float rho_new = d[0], rw = d[1], rr = d[2];
        const int it = st->iter + 1;
        st->iter = it;
        const float rec = sqrtf(rr);
        st->rec = rec;
        int reason = 0;
        const float alpha = st->alpha, omega = st->omega, rho = st->rho;
        const float bn = ((alpha / omega) * rho_new) / rho;
        const float den = (rw + bn * st->rs) - (bn * omega) * st->rz;
        if (rho_new == 0.0f || den == 0.0f || !isfinite(den)) reason |= R_BREAKDOWN;
        else { st->beta = bn; st->alpha = rho_new / den; st->rho = rho_new; }
        if (rec <= st->lim) reason |= R_CONVERGED;
        if (rec <= st->tol) reason |= R_CHECK;
        if (rec < st->best) { st->best = rec; st->it_best = it; }
        else if (st->stall > 0 && it - st->it_best >= st->stall) reason |= R_STALL;
        if (it >= st->max_iter) reason |= R_MAXIT;
        if (reason) { st->halt = 1; st->reason |= reason; }
    }
};

}  // namespace pbcg
