// Exact dot-product engine for gfx950 (wave64).
//
// What it computes: RN_even(sum_i x_i*y_i) with the sum formed exactly, the
// reproducible-reduction idea the paper borrows from ExBLAS (Section 2, the
// paragraph on the pure-MPI reproducible BiCGStab): a long fixed-point
// accumulator plus floating-point expansions, so that the rounded result is
// independent of partitioning, order and reduction tree.
//
// Representation.  Every product of two doubles is an integer multiple of
// 2^-2148, so the exact sum is S * 2^-2148 for an integer S with |S| < 2^4240.
// S is held as NCH = 132 signed 64-bit "chunks": chunk c carries weight 2^(32c);
// a chunk may exceed 32 bits (the upper half is carry headroom), so additions need
// no carry propagation until the end.
//
// Three levels:
//  1. Per lane: each product p = fl(x*y) and its exact error e = fma(x,y,-p)
//     (TwoProd, exact whenever 2^-969 <= |p| < 2^980) are added into a K-term
//     floating-point expansion with Knuth's TwoSum (error-free).  A non-zero
//     remainder after the K-th term, and every product outside the TwoProd range
//     (tiny, huge, or underflowed to zero), is deposited into the LDS accumulator
//     as an exact integer (ds_add_u64 atomics; integer adds commute).  The standalone dot
//     queues the out-of-range products per wave and deposits them 64 at a time.
//  2. Per wave at the end of the loop: each expansion term is summed exactly over
//     the 64 lanes inside a 4-chunk window (FP64 sums of integers < 2^38 are exact)
//     and one lane deposits the 4 window chunks; lanes outside the window deposit
//     their own term.
//  3. Per block: the LDS accumulator is carry-normalised one step (chunks become
//     |c| < 2^32 + 2^30) and its non-zero chunk range written to a per-block record;
//     a one-block finalize kernel, launched after the producer, sums the records
//     chunk by chunk (int64, order-free), normalises and rounds once to nearest-even.
// Integer addition is associative, so the bits of the result do not depend on the
// grid, the block size, K, or the order in which blocks finish.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xd {

constexpr int NCH = 132;     // chunks: bits 0 .. 4223 (+ 32 bits headroom in the top chunk)
constexpr int BIAS = 2148;   // bit k of S has weight 2^(k - 2148)
constexpr int WAVE = 64;

enum : uint32_t { F_NAN = 1u, F_PINF = 2u, F_NINF = 4u };

// Per-block record in global memory: header + chunk values [lo, hi].
struct RecHdr {
    int32_t lo, hi;
    uint32_t flags;
    int32_t pad;
};

// Workspace of one dot "site" (a kernel that produces D dots).
struct Site {
    RecHdr* hdr;           // [grid][D]
    long long* dig;        // [grid][D][NCH]
};

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

// value = m * 2^(P - BIAS), m < 2^53
__device__ __forceinline__ void decompose(double v, uint64_t& m, int& P, bool& neg) {
    uint64_t b = dbits(v);
    neg = (b >> 63) != 0;
    int be = (int)((b >> 52) & 0x7ff);
    m = b & ((1ull << 52) - 1);
    if (be) {
        m |= (1ull << 52);
        P = be - 1075 + BIAS;
    } else {
        P = -1074 + BIAS;
    }
}

__device__ __forceinline__ void lds_add(unsigned long long* acc, int c, uint64_t piece, bool neg) {
    if (piece) {
        long long v = neg ? -(long long)piece : (long long)piece;
        atomicAdd(acc + c, (unsigned long long)v);
    }
}

// Deposit a finite non-zero double exactly.
__device__ __forceinline__ void deposit_double(unsigned long long* acc, double v) {
    uint64_t m; int P; bool neg;
    decompose(v, m, P, neg);
    int c = P >> 5, s = P & 31;
    uint64_t lo = m << s;
    uint64_t hi = s ? (m >> (64 - s)) : 0;
    const long long sg = neg ? -1 : 1;
    atomicAdd(acc + c, (unsigned long long)(sg * (long long)(lo & 0xffffffffull)));
    atomicAdd(acc + c + 1, (unsigned long long)(sg * (long long)(lo >> 32)));
    if (hi) atomicAdd(acc + c + 2, (unsigned long long)(sg * (long long)hi));
}

// Deposit the exact product of two finite non-zero doubles (any magnitudes).
__device__ __forceinline__ void deposit_product(unsigned long long* acc, double x, double y) {
    uint64_t mx, my; int Px, Py; bool nx, ny;
    decompose(x, mx, Px, nx);
    decompose(y, my, Py, ny);
    uint64_t lo = mx * my;
    uint64_t hi = __umul64hi(mx, my);       // product < 2^106
    int P = Px + Py - BIAS;                  // >= 0
    int c = P >> 5, s = P & 31;
    uint64_t w0 = lo << s;
    uint64_t w1 = s ? ((hi << s) | (lo >> (64 - s))) : hi;
    uint64_t w2 = s ? (hi >> (64 - s)) : 0;
    bool neg = nx != ny;
    lds_add(acc, c, w0 & 0xffffffffull, neg);
    lds_add(acc, c + 1, w0 >> 32, neg);
    lds_add(acc, c + 2, w1 & 0xffffffffull, neg);
    lds_add(acc, c + 3, w1 >> 32, neg);
    lds_add(acc, c + 4, w2, neg);
}

// Knuth TwoSum: s + err == a + b exactly (no overflow).
__device__ __forceinline__ double two_sum(double a, double b, double& err) {
    double s = a + b;
    double bp = s - a;
    double ap = s - bp;
    err = (a - ap) + (b - bp);
    return s;
}

// Add v into expansion terms e[start..K-1]; a non-zero remainder goes to LDS.
template <int K>
__device__ __forceinline__ void expand(double (&e)[K], double v, int start, unsigned long long* acc) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k >= start) e[k] = two_sum(e[k], v, v);
    }
    if (v != 0.0) deposit_double(acc, v);
}

// Accumulate x*y exactly.  flags: block-shared non-finite flags.
template <int K>
__device__ __forceinline__ void accumulate(double (&e)[K], double x, double y,
                                           unsigned long long* acc, uint32_t* flags) {
    double p = x * y;
    int pe = (int)((dbits(p) >> 52) & 0x7ff);
    if (pe >= 54 && pe <= 2002) {            // 2^-969 <= |p| < 2^980: TwoProd is exact
        double err = fma(x, y, -p);
        expand<K>(e, p, 0, acc);
        expand<K>(e, err, K > 1 ? 1 : 0, acc);
    } else {
        bool fx = isfinite(x), fy = isfinite(y);
        if (!(fx && fy)) {
            uint32_t f;
            if (isnan(x) || isnan(y) || x == 0.0 || y == 0.0) f = F_NAN;
            else f = ((x > 0.0) == (y > 0.0)) ? F_PINF : F_NINF;
            atomicOr(flags, f);
        } else if (x != 0.0 && y != 0.0) {
            deposit_product(acc, x, y);      // tiny, underflowed or huge product
        }
    }
}

// Accumulate x*y exactly, with the rare products outside TwoProd's exact range queued per
// wave instead of deposited by the few lanes that meet them: the active lanes append them
// to the wave's LDS queue (qx, qy: 128 entries, compaction by ballot; *qn, in LDS, counts
// them), and once 64 are queued the active lanes deposit those 64 between them.  Any set
// of active lanes may call it (a wave's last trip can be partial); every lane of the wave
// must have the same qx, qy, qn.  drain_queue deposits what is left.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    const int lane = threadIdx.x & 63;
    return __popcll(lane ? (m << (64 - lane)) : 0ull);
}

template <int K>
__device__ __forceinline__ void accumulate_q(double (&e)[K], double x, double y, unsigned long long* acc,
                                             uint32_t* flags, double* qx, double* qy, int* qn) {
    double p = x * y;
    int pe = (int)((dbits(p) >> 52) & 0x7ff);
    bool queue = false;
    if (pe >= 54 && pe <= 2002) {
        double err = fma(x, y, -p);
        expand<K>(e, p, 0, acc);
        expand<K>(e, err, K > 1 ? 1 : 0, acc);
    } else {
        bool fx = isfinite(x), fy = isfinite(y);
        if (!(fx && fy)) {
            uint32_t f;
            if (isnan(x) || isnan(y) || x == 0.0 || y == 0.0) f = F_NAN;
            else f = ((x > 0.0) == (y > 0.0)) ? F_PINF : F_NINF;
            atomicOr(flags, f);
        } else if (x != 0.0 && y != 0.0) {
            queue = true;
        }
    }
    const uint64_t qm = __ballot(queue);
    if (qm) {
        int n = *qn;
        if (queue) {
            const int pos = n + lanes_below(qm);
            qx[pos] = x;
            qy[pos] = y;
        }
        n += __popcll(qm);
        if (n >= 64) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const uint64_t act = __ballot(true);
            const int nact = __popcll(act);
            for (int j = lanes_below(act); j < 64; j += nact) deposit_product(acc, qx[n - 64 + j], qy[n - 64 + j]);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            n -= 64;
        }
        *qn = n;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

__device__ __forceinline__ void drain_queue(unsigned long long* acc, const double* qx, const double* qy,
                                            const int* qn) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int n = *qn;
    const int lane = threadIdx.x & 63;
    if (lane < n) deposit_product(acc, qx[lane], qy[lane]);
}

// Cross-lane moves within a row of 16 lanes (DPP, register to register): quad_perm
// [1,0,3,2] and [2,3,0,1] exchange with lane^1 and lane^2, row_ror:4 and row_ror:8
// rotate the row.  Applied in that order, a + move(a) leaves every lane of the row
// holding the row's total.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = dpp_move<CTRL>(__double2loint(v));
    const int hi = dpp_move<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_ROR4 = 0x124, DPP_ROR8 = 0x128;

__device__ __forceinline__ int row_min_i(int v) {
    v = min(v, dpp_move<DPP_XOR1>(v));
    v = min(v, dpp_move<DPP_XOR2>(v));
    v = min(v, dpp_move<DPP_ROR4>(v));
    v = min(v, dpp_move<DPP_ROR8>(v));
    return v;
}

__device__ __forceinline__ double row_sum_d(double v) {
    v = v + dpp_move<DPP_XOR1>(v);
    v = v + dpp_move<DPP_XOR2>(v);
    v = v + dpp_move<DPP_ROR4>(v);
    v = v + dpp_move<DPP_ROR8>(v);
    return v;
}

// Exact deposit of one double per lane (zeros ignored), reduced per row of 16 lanes.
// All 64 lanes of the wave must call it together.  In each round, the row's pending
// values whose 32-bit chunk index is within one of the smallest pending index are cut
// at that chunk into four signed 32-bit pieces; the pieces are summed across the row
// in FP64 (at most 16 integers below 2^32: exact) and the row's leader adds the four
// sums into the accumulator.  The lane holding the smallest index always joins, so a
// row needs at most 16 rounds; typically one or two.
__device__ __forceinline__ void wave_deposit(unsigned long long* acc, double v) {
    bool pending = v != 0.0;
    if (__ballot(pending) == 0) return;
    uint64_t m = 0; int P = 0; bool neg = false;
    if (pending) decompose(v, m, P, neg);
    const int c = pending ? (P >> 5) : 0x7fffffff;
    while (__ballot(pending) != 0) {
        const int cmin = row_min_i(pending ? c : 0x7fffffff);
        const bool inwin = pending && (c - cmin) <= 1;
        double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
        if (inwin) {
            int sh = P - 32 * cmin;                 // 0..63
            uint64_t w0 = m << sh;
            uint64_t w1 = sh ? (m >> (64 - sh)) : 0;
            double sg = neg ? -1.0 : 1.0;
            q0 = sg * (double)(w0 & 0xffffffffull);
            q1 = sg * (double)(w0 >> 32);
            q2 = sg * (double)(w1 & 0xffffffffull);
            q3 = sg * (double)(w1 >> 32);
        }
        q0 = row_sum_d(q0);
        q1 = row_sum_d(q1);
        q2 = row_sum_d(q2);
        q3 = row_sum_d(q3);
        if ((threadIdx.x & 15) == 0 && cmin != 0x7fffffff) {
            if (q0 != 0.0) atomicAdd(acc + cmin, (unsigned long long)(long long)q0);
            if (q1 != 0.0) atomicAdd(acc + cmin + 1, (unsigned long long)(long long)q1);
            if (q2 != 0.0) atomicAdd(acc + cmin + 2, (unsigned long long)(long long)q2);
            if (q3 != 0.0 && cmin + 3 < NCH) atomicAdd(acc + cmin + 3, (unsigned long long)(long long)q3);
        }
        pending = pending && !inwin;
    }
}

// ------------------------------------------------------------------------------
// Block-level protocol.  `acc` is __shared__ unsigned long long[D*NCH], `flags`
// __shared__ uint32_t[D]; both zeroed by block_init before the loop.
template <int D>
__device__ __forceinline__ void block_init(unsigned long long* acc, uint32_t* flags) {
    for (int i = threadIdx.x; i < D * NCH; i += blockDim.x) acc[i] = 0ull;
    if (threadIdx.x < D) flags[threadIdx.x] = 0u;
    __syncthreads();
}

// Flush every lane's expansions (all threads of the block call this).
template <int D, int K>
__device__ __forceinline__ void block_flush(double (&e)[D][K], unsigned long long* acc) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int k = 0; k < K; ++k) wave_deposit(acc + d * NCH, e[d][k]);
    }
    __syncthreads();
}

// Write this block's record (one-step carry normalisation, non-zero range).
// `tmp` is __shared__ long long[D*NCH] scratch, `rng` __shared__ int[2*D].
template <int D>
__device__ void block_write(const Site& site, unsigned long long* acc, uint32_t* flags,
                            long long* tmp, int* rng) {
    const int tid = threadIdx.x;
    if (tid < D) { rng[2 * tid] = NCH; rng[2 * tid + 1] = -1; }
    // balanced split: a = lo + 2^32 hi with lo in [-2^31, 2^31)
    for (int i = tid; i < D * NCH; i += blockDim.x) {
        long long a = (long long)acc[i];
        int c = i % NCH;
        long long hi = (c == NCH - 1) ? 0 : ((a - (long long)(int32_t)(uint32_t)a) >> 32);
        tmp[i] = hi;
    }
    __syncthreads();
    for (int i = tid; i < D * NCH; i += blockDim.x) {
        long long a = (long long)acc[i];
        int c = i % NCH, d = i / NCH;
        long long lo = (c == NCH - 1) ? a : (long long)(int32_t)(uint32_t)a;
        long long v = lo + (c > 0 ? tmp[i - 1] : 0);
        acc[i] = (unsigned long long)v;
        if (v != 0) {
            atomicMin(&rng[2 * d], c);
            atomicMax(&rng[2 * d + 1], c);
        }
    }
    __syncthreads();
    const size_t b = blockIdx.x;
    for (int i = tid; i < D * NCH; i += blockDim.x) {
        int c = i % NCH, d = i / NCH;
        if (c >= rng[2 * d] && c <= rng[2 * d + 1])
            site.dig[(b * D + d) * NCH + c] = (long long)acc[i];
    }
    if (tid < D) {
        RecHdr h;
        h.lo = rng[2 * tid];
        h.hi = rng[2 * tid + 1];
        h.flags = flags[tid];
        h.pad = 0;
        site.hdr[b * D + tid] = h;
    }
}

// Round S * 2^-2148 to FP64, nearest-even.  s[0..NCH-1] holds chunk sums (destroyed);
// only chunks in [lo, hi] are non-zero on entry (lo > hi: S = 0).
__device__ double round_chunks(long long* s, uint32_t flags, int lo, int hi) {
    if ((flags & F_NAN) || ((flags & F_PINF) && (flags & F_NINF))) return __longlong_as_double(0x7ff8000000000000ll);
    if (flags & F_PINF) return __longlong_as_double(0x7ff0000000000000ll);
    if (flags & F_NINF) return __longlong_as_double((long long)0xfff0000000000000ull);
    if (lo > hi) return 0.0;
    // balanced normalisation: digits in [-2^31, 2^31); carries stop a few chunks above hi
    long long carry = 0;
    int c = lo;
    for (; c < NCH - 1 && (c <= hi || carry != 0); ++c) {
        long long v = s[c] + carry;
        long long d = (long long)(int32_t)(uint32_t)v;
        carry = (v - d) >> 32;
        s[c] = d;
    }
    if (carry != 0) s[c] += carry;      // c == NCH - 1: the top chunk keeps the excess
    int top = -1;
    for (int k = c; k >= lo; --k) {
        if (s[k] != 0) { top = k; break; }
    }
    if (top < 0) return 0.0;            // exact zero -> +0
    const bool neg = s[top] < 0;
    // magnitude in standard digits [0, 2^32) (a borrow can only shrink the top)
    carry = 0;
    for (int k = lo; k <= top; ++k) {
        long long v = (neg ? -s[k] : s[k]) + carry;
        if (k == NCH - 1) { s[k] = v; break; }
        long long d = v & 0xffffffffll;
        carry = (v - d) >> 32;
        s[k] = d;
    }
    int h = -1;
    for (int k = top; k >= lo; --k) {
        if (s[k] != 0) { h = k; break; }
    }
    const uint64_t sign = neg ? 0x8000000000000000ull : 0ull;
    if (h >= 100) return __longlong_as_double((long long)(sign | 0x7ff0000000000000ull));  // >= 2^1052
    const int msb = 32 * h + 31 - __clz((unsigned int)s[h]);
    const int cut = max(msb - 52, 1074);           // bit index of the last place
    auto dig = [&](int k) -> uint64_t { return (k >= lo && k <= h) ? (uint64_t)s[k] : 0ull; };
    auto get64 = [&](int off) -> uint64_t {
        int k = off >> 5, sh = off & 31;
        uint64_t w = dig(k) | (dig(k + 1) << 32);
        uint64_t r = w >> sh;
        if (sh) r |= dig(k + 2) << (64 - sh);
        return r;
    };
    uint64_t mant = get64(cut) & ((1ull << 53) - 1);
    const int g = cut - 1;
    uint64_t guard = get64(g) & 1ull;
    bool sticky = false;
    {
        int k = g >> 5, sh = g & 31;
        for (int j = lo; j < k && j <= h; ++j) sticky |= (s[j] != 0);
        if (sh) sticky |= (dig(k) & ((1ull << sh) - 1)) != 0;
    }
    uint64_t bits = ((uint64_t)(cut - 1074) << 52) + mant;
    if (guard && (sticky || (mant & 1ull))) bits += 1;
    if (bits >= 0x7ff0000000000000ull) bits = 0x7ff0000000000000ull;
    return __longlong_as_double((long long)(sign | bits));
}

// Sum the G per-block records of D dots and round each (one block, run by the
// finalize kernel after the producer kernel has completed).  `fin` is __shared__
// long long[D*NCH], `hlo/hhi` __shared__ short[G_MAX*D], `fl` uint32_t[D], `rng`
// int[2D]; the D results land in out[] (shared), valid after the final barrier.
template <int D, int GMAX>
__device__ void reduce_records(const Site& site, int G, long long* fin, short* hlo, short* hhi,
                               uint32_t* fl, int* rng, double* out) {
    const int tid = threadIdx.x;
    for (int i = tid; i < D * NCH; i += blockDim.x) fin[i] = 0;
    if (tid < D) { fl[tid] = 0u; rng[2 * tid] = NCH; rng[2 * tid + 1] = -1; }
    __syncthreads();
    // headers: every load of a thread is issued before the first use (one round of memory
    // latency instead of one per header); HB covers G * D <= GMAX * D with 1024 threads
    constexpr int HB = (GMAX * D) / 1024 < 1 ? 1 : ((GMAX * D) / 1024 > 8 ? 8 : (GMAX * D) / 1024);
    for (int j0 = tid; j0 < G * D; j0 += HB * blockDim.x) {
        RecHdr h[HB];
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int j = j0 + u * blockDim.x;
            if (j < G * D) h[u] = site.hdr[j];
        }
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int j = j0 + u * blockDim.x;
            if (j < G * D) {
                hlo[j] = (short)h[u].lo;
                hhi[j] = (short)h[u].hi;
                const int d = j % D;
                if (h[u].flags) atomicOr(&fl[d], h[u].flags);
                if (h[u].lo <= h[u].hi) {
                    atomicMin(&rng[2 * d], h[u].lo);
                    atomicMax(&rng[2 * d + 1], h[u].hi);
                }
            }
        }
    }
    __syncthreads();
    // all dots in one pass: item j -> (dot d, record g, chunk c) over the union of windows
    int off[D + 1], LOd[D], Wd[D];
    off[0] = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        LOd[d] = rng[2 * d];
        Wd[d] = rng[2 * d + 1] >= rng[2 * d] ? rng[2 * d + 1] - rng[2 * d] + 1 : 0;
        off[d + 1] = off[d] + G * Wd[d];
    }
    const int items = off[D];
    constexpr int U = 8;    // with the finalize kernel's 1024 threads: 8192 chunk loads per round
    for (int j0 = tid; j0 < items; j0 += U * blockDim.x) {
        long long v[U];
        int slot[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * blockDim.x;
            v[u] = 0;
            slot[u] = -1;
            if (j < items) {
                int d = 0;
#pragma unroll
                for (int e = 1; e < D; ++e) d += (j >= off[e]) ? 1 : 0;
                const int jj = j - off[d];
                const int gg = jj / Wd[d], c = LOd[d] + jj % Wd[d];
                const int hj = gg * D + d;
                if (c >= hlo[hj] && c <= hhi[hj]) {
                    v[u] = site.dig[(size_t)hj * NCH + c];
                    slot[u] = d * NCH + c;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (slot[u] >= 0 && v[u] != 0) atomicAdd((unsigned long long*)&fin[slot[u]], (unsigned long long)v[u]);
    }
    __syncthreads();
    if (tid < D) out[tid] = round_chunks(fin + tid * NCH, fl[tid], rng[2 * tid], rng[2 * tid + 1]);
    __syncthreads();
}

}  // namespace xd
