// Learned sparse approximate inverse on A's pattern: feature, MLP (FP32 training and
// bf16-MFMA inference), probe products, loss / gradient and Adam kernels (gfx950).
//
// m_ij = ([i = j] + f(phi_ij)) / a_ii,  f: 12 -> 64 -> 64 -> 1 with GELU (erf form);
// loss L = ||M U - V||_F^2 / (k n) with U = A V for probe blocks V (n x k).
// Deterministic by construction: no floating-point atomics; every reduction runs in a
// fixed order (column sums of |A| use exact fixed-point integer atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/pbicgstab.h"

#pragma clang fp contract(off)

namespace {

constexpr int NF = 12, HID = 64;
constexpr int NPARAM = HID * NF + HID + HID * HID + HID + HID + 1;  // 5057
constexpr int OFF_W1 = 0, OFF_B1 = HID * NF, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
constexpr int BLOCK = 256;
constexpr int GRAD_BLOCKS = 256;   // fixed partition of the weight-gradient reduction
constexpr int ACT = 4 * HID + 1;   // per-nonzero saved values: dz1, h1, dz2, h2, g_f

#define HIPCHK(expr)                              \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return PBCG_ERR_HIP; \
    } while (0)

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = expf(-0.5f * x * x) * 0.39894228040143268f;
    return cdf + x * pdf;
}

// ------------------------------------------------------------------ matrix statistics
__global__ void k_zero64(unsigned long long* p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// maximum |a| as its bit pattern (positive doubles order like their bits)
__global__ void __launch_bounds__(BLOCK) k_maxabs(int64_t nnz, const double* __restrict__ val,
                                                  unsigned long long* out) {
    unsigned long long m = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (unsigned long long)__double_as_longlong(fabs(val[k])));
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned long long)__shfl_xor((long long)m, o));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

struct Stats {
    double* diag;              // a_ii (0 if absent)
    double* rsum;              // sum_j |a_ij|, left to right
    unsigned long long* cfix;  // sum_i |a_ij| as a fixed-point integer (scale 2^cshift)
    float* maxoff;             // max_{j in row i} |j - i|
    int* maxlen;               // max row length
    int* rowidx;               // row of every nonzero
};

__global__ void __launch_bounds__(BLOCK) k_row_stats(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                     const double* __restrict__ val, const unsigned long long* maxabs_bits,
                                                     Stats st) {
    // fixed-point scale: n * max|a| * 2^s < 2^62
    const double maxabs = __longlong_as_double((long long)*maxabs_bits);
    int e = 0;
    frexp(maxabs * (double)max(n, 1), &e);
    const int cshift = 61 - e;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], b = rp[i + 1];
    double r = 0.0, d = 0.0;
    int mo = 0;
    for (int k = a; k < b; ++k) {
        const int j = ci[k];
        const double v = val[k];
        r = r + fabs(v);
        if (j == i) d = v;
        mo = max(mo, abs(j - i));
        st.rowidx[k] = i;
        const unsigned long long q = (unsigned long long)llrint(ldexp(fabs(v), cshift));
        atomicAdd(st.cfix + j, q);   // integer sums commute: deterministic
    }
    st.diag[i] = d;
    st.rsum[i] = r;
    st.maxoff[i] = (float)mo;
    atomicMax(st.maxlen, b - a);
}

__device__ __forceinline__ double col_sum(const Stats& st, int j, int cshift) {
    return ldexp((double)st.cfix[j], -cshift);
}

// a_ji by binary search in row j (columns ascending); 0 if absent
__device__ __forceinline__ double lookup(const int32_t* rp, const int32_t* ci, const double* val, int j, int i) {
    int lo = rp[j], hi = rp[j + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = ci[mid];
        if (c == i) return val[mid];
        if (c < i) lo = mid + 1;
        else hi = mid - 1;
    }
    return 0.0;
}

__global__ void __launch_bounds__(BLOCK) k_features(int n, int64_t nnz, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                    Stats st, const unsigned long long* maxabs_bits,
                                                    float* __restrict__ feat) {
    const double maxabs = __longlong_as_double((long long)*maxabs_bits);
    int e = 0;
    frexp(maxabs * (double)max(n, 1), &e);
    const int cshift = 61 - e;
    const double maxlen = (double)*st.maxlen;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
        const int i = st.rowidx[k], j = ci[k];
        const double aij = val[k];
        const double aji = lookup(rp, ci, val, j, i);
        const double dii = st.diag[i], djj = st.diag[j];
        const double adi = fabs(dii), adj = fabs(djj);
        const double mo = (double)st.maxoff[i];
        float* f = feat + k * NF;
        f[0] = (float)(aij / adi);
        f[1] = (float)(aji / adi);
        f[2] = (float)(djj / adi);
        f[3] = (float)((dii > 0.0) - (dii < 0.0));
        f[4] = (float)(st.rsum[i] / adi);
        f[5] = (float)(st.rsum[j] / adj);
        f[6] = (float)(col_sum(st, i, cshift) / adi);
        f[7] = (float)(col_sum(st, j, cshift) / adj);
        f[8] = (float)((double)(rp[i + 1] - rp[i]) / maxlen);
        f[9] = mo > 0.0 ? (float)((double)(j - i) / mo) : 0.0f;
        f[10] = i == j ? 1.0f : 0.0f;
        const double den = fmax(fabs(aij + aji), 0x1p-126);
        f[11] = i == j ? 0.0f : (float)(fabs(aij - aji) / den);
    }
}

// ------------------------------------------------------------------ FP32 MLP
struct SmemW {
    float W1[HID * NF], b1[HID], W2[HID * HID], b2[HID], w3[HID], b3;
};

__device__ __forceinline__ void load_weights(SmemW& s, const float* p) {
    for (int t = threadIdx.x; t < NPARAM; t += blockDim.x) ((float*)&s)[t] = p[t];
    __syncthreads();
}

// forward of one nonzero; keeps z1 and z2 (pre-activations) for the backward
__device__ __forceinline__ float mlp_forward(const SmemW& s, const float* x, float* z1, float* z2) {
    float h1[HID];
#pragma unroll 4
    for (int a = 0; a < HID; ++a) {
        float acc = s.b1[a];
#pragma unroll
        for (int c = 0; c < NF; ++c) acc = acc + s.W1[a * NF + c] * x[c];
        z1[a] = acc;
        h1[a] = gelu(acc);
    }
    float f = s.b3;
    for (int a = 0; a < HID; ++a) {
        float acc = s.b2[a];
#pragma unroll 8
        for (int b = 0; b < HID; ++b) acc = acc + s.W2[a * HID + b] * h1[b];
        z2[a] = acc;
        f = f + s.w3[a] * gelu(acc);
    }
    return f;
}

__global__ void __launch_bounds__(BLOCK) k_forward(int64_t nnz, const float* __restrict__ feat, const float* __restrict__ params,
                                                   const int* __restrict__ rowidx,
                                                   const double* __restrict__ diag, float* __restrict__ fout,
                                                   float* __restrict__ mout) {
    __shared__ SmemW s;
    load_weights(s, params);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
        float x[NF], z1[HID], z2[HID];
#pragma unroll
        for (int c = 0; c < NF; ++c) x[c] = feat[k * NF + c];
        const float f = mlp_forward(s, x, z1, z2);
        if (fout) fout[k] = f;
        const int i = rowidx[k];
        mout[k] = (x[10] + f) / (float)diag[i];
    }
}

// ------------------------------------------------------------------ probe products
// U = A V  (FP64 values, FP32 probes; row sums left to right in FP64, stored FP32)
__global__ void __launch_bounds__(BLOCK) k_probe_product(int n, int k, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                         const float* __restrict__ V, float* __restrict__ U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < k; ++c) {
        double s = 0.0;
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            double prod = val[q] * (double)V[(size_t)c * n + ci[q]];
            s = s + prod;
        }
        U[(size_t)c * n + i] = (float)s;
    }
}

// R = M U - V (FP32, M values on A's pattern), plus per-block partial sums of R^2
__global__ void __launch_bounds__(BLOCK) k_residual(int n, int k, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const float* __restrict__ m,
                                                    const float* __restrict__ U, const float* __restrict__ V,
                                                    float* __restrict__ R, float* __restrict__ part) {
    __shared__ float red[BLOCK];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.0f;
    if (i < n) {
        for (int c = 0; c < k; ++c) {
            float s = 0.0f;
            for (int q = rp[i]; q < rp[i + 1]; ++q) {
                float prod = m[q] * U[(size_t)c * n + ci[q]];
                s = s + prod;
            }
            const float r = s - V[(size_t)c * n + i];
            R[(size_t)c * n + i] = r;
            float r2 = r * r;
            sq = sq + r2;
        }
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = (sum of block partials in block order) / (k n)
__global__ void k_loss(int nb, const float* part, float scale, float* loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int b = 0; b < nb; ++b) s = s + part[b];
        *loss = s * scale;
    }
}

// per nonzero: g_m = scale * sum_c R_ic U_jc (SDDMM), g_f = g_m / a_ii, then the MLP
// backward; saves dz1, h1, dz2, h2, g_f for the weight-gradient reduction
__global__ void __launch_bounds__(BLOCK) k_backward(int n, int64_t nnz, int k, const float* __restrict__ feat,
                                                    const float* __restrict__ params, const int* __restrict__ rowidx,
                                                    const int32_t* __restrict__ ci, const double* __restrict__ diag,
                                                    const float* __restrict__ R, const float* __restrict__ U, float scale,
                                                    float* __restrict__ act) {
    __shared__ SmemW s;
    load_weights(s, params);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = rowidx[q], j = ci[q];
        float gm = 0.0f;
        for (int c = 0; c < k; ++c) {
            float prod = R[(size_t)c * n + i] * U[(size_t)c * n + j];
            gm = gm + prod;
        }
        gm = gm * scale;
        const float gf = gm / (float)diag[i];
        float x[NF], z1[HID], z2[HID];
#pragma unroll
        for (int c = 0; c < NF; ++c) x[c] = feat[q * NF + c];
        (void)mlp_forward(s, x, z1, z2);
        float* o = act + q * ACT;
        float dz2[HID];
        for (int a = 0; a < HID; ++a) {
            float t = gf * s.w3[a];
            dz2[a] = t * gelu_grad(z2[a]);
            o[2 * HID + a] = dz2[a];
            o[3 * HID + a] = gelu(z2[a]);
        }
        for (int b = 0; b < HID; ++b) {
            float dh = 0.0f;
#pragma unroll 8
            for (int a = 0; a < HID; ++a) dh = dh + s.W2[a * HID + b] * dz2[a];
            o[b] = dh * gelu_grad(z1[b]);
            o[HID + b] = gelu(z1[b]);
        }
        o[4 * HID] = gf;
    }
}

// gradient entry e of a nonzero's contribution (x = features, saved activations a)
__device__ __forceinline__ float grad_term(int e, const float* x, const float* a) {
    if (e < OFF_B1) return a[e / NF] * x[e % NF];                         // dW1 = dz1 (x) phi
    if (e < OFF_W2) return a[e - OFF_B1];                                  // db1 = dz1
    if (e < OFF_B2) { int t = e - OFF_W2; return a[2 * HID + t / HID] * a[HID + t % HID]; }  // dW2 = dz2 (x) h1
    if (e < OFF_W3) return a[2 * HID + (e - OFF_B2)];                      // db2 = dz2
    if (e < OFF_B3) return a[4 * HID] * a[3 * HID + (e - OFF_W3)];         // dw3 = g_f h2
    return a[4 * HID];                                                     // db3 = g_f
}

// block b sums the contributions of nonzeros [b*C, (b+1)*C) in order; tiles of 16
// nonzeros are staged in LDS
constexpr int TILE = 16;
__global__ void __launch_bounds__(BLOCK) k_grad_partial(int64_t nnz, const float* __restrict__ feat,
                                                        const float* __restrict__ act, float* __restrict__ part) {
    __shared__ float sx[TILE][NF];
    __shared__ float sa[TILE][ACT];
    constexpr int PER = (NPARAM + BLOCK - 1) / BLOCK;   // 20 entries per thread
    float acc[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) acc[u] = 0.0f;
    const int64_t C = (nnz + gridDim.x - 1) / gridDim.x;
    const int64_t k0 = (int64_t)blockIdx.x * C, k1 = min(nnz, k0 + C);
    for (int64_t t0 = k0; t0 < k1; t0 += TILE) {
        const int cnt = (int)min((int64_t)TILE, k1 - t0);
        for (int z = threadIdx.x; z < TILE * NF; z += blockDim.x) {
            const int r = z / NF, c = z % NF;
            sx[r][c] = r < cnt ? feat[(t0 + r) * NF + c] : 0.0f;
        }
        for (int z = threadIdx.x; z < TILE * ACT; z += blockDim.x) {
            const int r = z / ACT, c = z % ACT;
            sa[r][c] = r < cnt ? act[(t0 + r) * ACT + c] : 0.0f;
        }
        __syncthreads();
        for (int r = 0; r < cnt; ++r) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = threadIdx.x + u * BLOCK;
                if (e < NPARAM) {
                    float v = grad_term(e, sx[r], sa[r]);
                    acc[u] = acc[u] + v;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * BLOCK;
        if (e < NPARAM) part[(size_t)blockIdx.x * NPARAM + e] = acc[u];
    }
}

__global__ void __launch_bounds__(BLOCK) k_grad_sum(int nb, const float* __restrict__ part, float* __restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPARAM) return;
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s = s + part[(size_t)b * NPARAM + e];
    grad[e] = s;
}

__global__ void __launch_bounds__(BLOCK) k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                                const float* __restrict__ g, int t, float lr, float b1, float b2,
                                                float eps) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPARAM) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float mh = me / (1.0f - powf(b1, (float)t));
    const float vh = ve / (1.0f - powf(b2, (float)t));
    p[e] = p[e] - lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------ probe columns
// out[i] = fp32(r_i / sqrt(rr)) with rr the exact (r, r) rounded once; zero column if rr = 0
__global__ void __launch_bounds__(BLOCK) k_probe_column(int n, const double* __restrict__ r,
                                                        const double* __restrict__ rr, float* __restrict__ out) {
    const double nrm = sqrt(*rr);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[i] = nrm > 0.0 ? (float)(r[i] / nrm) : 0.0f;
}

// ------------------------------------------------------------------ bf16 MFMA inference
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));


// GELU for inference by linear interpolation in a table of GT_N intervals of width 2^-8 on
// [-8, 8), held in LDS.  Entry k = (G(z_k), G(z_{k+1}) - G(z_k)) at the nodes z_k = -8 + k/256
// (exact in FP32), with G(z) = z Phi(z) from erfcf in FP32 (erfc keeps the negative tail's
// relative accuracy).  Interpolation error <= h^2/8 max|G''| = 2^-16/8 * 2 phi(0) ~ 1.5e-6;
// the table position t = 256 z + 2048, accumulated at that scale, is off by a few FP32 ulps
// of 2048, which moves z by a few 2^-21: both far below the bf16 rounding the result gets
// next.  The first interval is flat (slope 0), so every z below -8 gives G(-8) (|G| < 1e-14
// there); from 7.996 on the nodes carry G(z) = z exactly in FP32 (Phi = 1 - 7e-16), so the
// last interval's linear extension is G(z) = z for every larger z.  NaN stays NaN.  Per
// GELU: a clamp, two conversions, a subtraction, the address, one LDS read of 8 bytes and
// one FMA -- no transcendental on the hot path.
constexpr int GT_N = 4096;

__device__ __forceinline__ float gelu_ref(float z) {
    const float h = 0.5f * erfcf(fabsf(z) * 0.70710678118654752f);     // Phi(-|z|)
    return z * (z >= 0.0f ? 1.0f - h : h);
}

__device__ void gelu_table_init(float2* tab) {
    for (int k = threadIdx.x; k < GT_N; k += blockDim.x) {
        const float z0 = -8.0f + (float)k * (1.0f / 256.0f);
        const float g0 = gelu_ref(z0), g1 = gelu_ref(z0 + (1.0f / 256.0f));
        tab[k] = make_float2(g0, k == 0 ? 0.0f : g1 - g0);
    }
    __syncthreads();
}

// G(z) from the table position t = 256 z + 2048, which the inference MFMAs produce directly.
__device__ __forceinline__ float gelu_lookup(const float2* tab, float t) {
    const int k = (int)__builtin_amdgcn_fmed3f(t, 0.0f, (float)(GT_N - 1));   // one v_med3_f32
    const float2 e = tab[k];
    return fmaf(t - (float)k, e.y, e.x);
}

// One wave handles tiles of 16 nonzeros with v_mfma_f32_16x16x32_bf16 (lane l = 16 g + c
// holds A[c][8 g + j] and B[8 g + j][c], j = 0..7, and C[4 g + j][c], j = 0..3).  The
// nonzeros are the N dimension: layer 1 computes H1 (64 hidden x 16 nonzeros) = W1 Phi as
// four 16-row tiles (K = 12 features padded to 32); lane (g, c) then holds hidden units
// 16 mt + 4 g + j of nonzero c, which are exactly the B operand of layer 2 once the 64
// hidden units are ordered (per 32-unit k-step ks) as 16 (2 ks) + 4 g + j, then
// 16 (2 ks + 1) + 4 g + j -- so W2's columns are taken in that order and no value
// crosses lanes.  The biases enter as the accumulators' initial values.  Layer 3 (64 -> 1)
// sums each lane's 16 units with packed bf16 dot products (v_dot2_f32_bf16, FP32
// accumulation), then the four lane groups.
// The weights (A operands in each lane's layout), biases and w3 live in LDS next to the GELU
// table and are read where they are used, by volatile LDS loads that the compiler cannot
// hoist into registers: the kernel then needs 63 VGPRs, so eight waves per SIMD stay
// resident (the register-held form had 126 VGPRs and four waves).  Two 1,024-thread blocks
// (45 KB of LDS each) fill a CU.
constexpr int INFER_BLOCK = 1024;
template <class T> __device__ __forceinline__ T lds_load(const T* p) {
    return *(__attribute__((address_space(3))) const volatile T*)p;
}

__global__ void __launch_bounds__(INFER_BLOCK) __attribute__((amdgpu_waves_per_eu(8)))
k_infer_bf16(int64_t nnz, const float* __restrict__ feat,
                                                    const float* __restrict__ params, const int* __restrict__ rowidx,
                                                    const double* __restrict__ diag, float* __restrict__ mout) {
    // W1 (4 m-tiles, K padded to 32) and the column-permuted W2 (4 m-tiles x 2 k-steps),
    // rounded to bf16, per lane l = 16 g + c; biases and w3 in the C layout (unit
    // 16 mt + 4 g + j, the same for the 16 lanes of a group).  W1, W2 are stored times 256
    // (exact in bf16) and the biases as 256 b + 2048, so that the MFMAs yield the GELU table
    // position t = 256 z + 2048 of each pre-activation z.
    __shared__ float2 gtab[GT_N];
    __shared__ bf16x8 sw1[4][64], sw2[4][2][64];
    __shared__ floatx4 sb1[4][4], sb2[4][4];
    __shared__ bf16x2 sw3[4][4][2];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        const int mt = i >> 4, g = (i >> 2) & 3, j = i & 3, u = 16 * mt + 4 * g + j;
        sb1[mt][g][j] = fmaf(params[OFF_B1 + u], 256.0f, 2048.0f);
        sb2[mt][g][j] = fmaf(params[OFF_B2 + u], 256.0f, 2048.0f);
        sw3[mt][g][j >> 1][j & 1] = (__bf16)params[OFF_W3 + u];
    }
    for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) {
        const int mt = i >> 6, ln = i & 63, cc = ln & 15, gg = ln >> 4, row = 16 * mt + cc;
        bf16x8 w;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * gg + j;
            w[j] = (__bf16)(k < NF ? 256.0f * params[OFF_W1 + row * NF + k] : 0.0f);
        }
        sw1[mt][ln] = w;
        for (int ks = 0; ks < 2; ++ks) {
            for (int j = 0; j < 8; ++j) {
                const int unit = 16 * (2 * ks + (j >> 2)) + 4 * gg + (j & 3);
                w[j] = (__bf16)(256.0f * params[OFF_W2 + row * HID + unit]);
            }
            sw2[mt][ks][ln] = w;
        }
    }
    gelu_table_init(gtab);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int c = lane & 15, grp = lane >> 4;
    const float b3 = params[OFF_B3];
    const int64_t ntiles = (nnz + 15) / 16;
    constexpr int WAVES = INFER_BLOCK / 64;
    const int64_t wstride = (int64_t)gridDim.x * WAVES;
    for (int64_t tile = (int64_t)blockIdx.x * WAVES + wid; tile < ntiles; tile += wstride) {
        const int64_t q = tile * 16 + c;          // this lane's nonzero
        // layer 1: B = features of the tile's nonzeros, rows 8 grp .. 8 grp + 7 of K
        bf16x8 bx;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * grp + j;
            bx[j] = (__bf16)((q < nnz && k < NF) ? feat[q * NF + k] : 0.0f);
        }
        bf16x8 h1[2];
        for (int mt = 0; mt < 4; ++mt) {
            const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_load(&sw1[mt][lane]), bx, lds_load(&sb1[mt][grp]), 0, 0, 0);
            for (int j = 0; j < 4; j += 2) {   // two values per conversion instruction
                const f32x2 g2 = {gelu_lookup(gtab, acc[j]), gelu_lookup(gtab, acc[j + 1])};
                const bf16x2 h2 = __builtin_convertvector(g2, bf16x2);
                h1[mt >> 1][4 * (mt & 1) + j] = h2[0];
                h1[mt >> 1][4 * (mt & 1) + j + 1] = h2[1];
            }
        }
        // layer 2: B = H1 in the permuted unit order (k-step ks = m-tiles 2 ks, 2 ks + 1)
        float part = 0.0f;
        for (int mt = 0; mt < 4; ++mt) {
            floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_load(&sw2[mt][0][lane]), h1[0], lds_load(&sb2[mt][grp]), 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_load(&sw2[mt][1][lane]), h1[1], acc, 0, 0, 0);
            // layer 3: f = sum_u bf16(gelu(z2_u)) w3_u + b3
            for (int j = 0; j < 4; j += 2) {
                const f32x2 g2 = {gelu_lookup(gtab, acc[j]), gelu_lookup(gtab, acc[j + 1])};
                const bf16x2 r2 = __builtin_convertvector(g2, bf16x2);
                part = __builtin_amdgcn_fdot2_f32_bf16(r2, lds_load(&sw3[mt][grp][j >> 1]), part, false);
            }
        }
        part = part + __shfl_xor(part, 16);
        part = part + __shfl_xor(part, 32);
        if (grp == 0 && q < nnz) {
            const float f = part + b3;
            const float isd = feat[q * NF + 10];
            mout[q] = (isd + f) / (float)diag[rowidx[q]];
        }
    }
}

// ------------------------------------------------------------------ workspace
struct SpaiWs {
    unsigned long long* maxabs;
    int* maxlen;
    double* diag;
    double* rsum;
    unsigned long long* cfix;
    float* maxoff;
    float* part;      // loss partials [ceil(n/BLOCK)]
    float* gpart;     // gradient partials [GRAD_BLOCKS][NPARAM]
    float* R;         // n x k
    float* act;       // nnz x ACT
    float* mstep;     // nnz: M values of a training step
    float* gstep;     // NPARAM: gradient of a training step
    size_t need;
};

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }

SpaiWs carve(void* ws, int32_t n, int64_t nnz, int32_t k) {
    SpaiWs w{};
    char* b = (char*)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) { char* p = b ? b + o : nullptr; o += al(bytes); return p; };
    w.maxabs = (unsigned long long*)take(8);
    w.maxlen = (int*)take(8);
    w.diag = (double*)take(sizeof(double) * (size_t)std::max(n, 1));
    w.rsum = (double*)take(sizeof(double) * (size_t)std::max(n, 1));
    w.cfix = (unsigned long long*)take(8 * (size_t)std::max(n, 1));
    w.maxoff = (float*)take(4 * (size_t)std::max(n, 1));
    w.part = (float*)take(4 * (size_t)((n + BLOCK - 1) / BLOCK + 1));
    w.gpart = (float*)take(4 * (size_t)GRAD_BLOCKS * NPARAM);
    w.R = (float*)take(4 * (size_t)std::max(n, 1) * std::max(k, 1));
    w.act = (float*)take(4 * (size_t)std::max<int64_t>(nnz, 1) * ACT);
    w.mstep = (float*)take(4 * (size_t)std::max<int64_t>(nnz, 1));
    w.gstep = (float*)take(4 * (size_t)NPARAM);
    w.need = o;
    return w;
}

bool csr_f64_ok(const pbcg_csr* A) {
    return A && A->n > 0 && A->nnz > 0 && A->nnz < (int64_t(1) << 31) && A->row_ptr && A->col_idx && A->val &&
           A->val_type == PBCG_F64;
}

int grid_for(int64_t items) { return (int)std::max<int64_t>(1, std::min<int64_t>((items + BLOCK - 1) / BLOCK, 8192)); }

}  // namespace

extern "C" {

int spai_param_count(void) { return NPARAM; }

size_t spai_workspace_bytes(int32_t n, int64_t nnz, int32_t k) { return carve(nullptr, n, nnz, k).need + 256; }

int spai_features(const pbcg_csr* A, float* feat, int32_t* rowidx, double* diag, void* ws, size_t ws_bytes,
                  void* stream) {
    if (!csr_f64_ok(A) || !feat || !rowidx || !diag) return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < spai_workspace_bytes(A->n, A->nnz, 1) || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs w = carve(ws, A->n, A->nnz, 1);
    k_zero64<<<1, 64, 0, s>>>(w.maxabs, 1);
    k_zero64<<<1, 64, 0, s>>>((unsigned long long*)w.maxlen, 1);
    k_zero64<<<grid_for(A->n), BLOCK, 0, s>>>(w.cfix, A->n);
    const double* val = (const double*)A->val;
    k_maxabs<<<grid_for(A->nnz), BLOCK, 0, s>>>(A->nnz, val, w.maxabs);
    Stats st{diag, w.rsum, w.cfix, w.maxoff, w.maxlen, rowidx};
    k_row_stats<<<(A->n + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(A->n, A->row_ptr, A->col_idx, val, w.maxabs, st);
    k_features<<<grid_for(A->nnz), BLOCK, 0, s>>>(A->n, A->nnz, A->row_ptr, A->col_idx, val, st, w.maxabs, feat);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int spai_forward(int64_t nnz, const float* feat, const float* params, const int32_t* rowidx, const int32_t* col_idx,
                 const double* diag, float* f_out, float* m_out, void* stream) {
    if (nnz <= 0 || !feat || !params || !rowidx || !col_idx || !diag || !m_out) return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    k_forward<<<grid_for(nnz), BLOCK, 0, s>>>(nnz, feat, params, rowidx, diag, f_out, m_out);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int spai_infer_bf16(int64_t nnz, const float* feat, const float* params, const int32_t* rowidx, const double* diag,
                    float* m_out, void* stream) {
    if (nnz <= 0 || !feat || !params || !rowidx || !diag || !m_out) return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const int64_t tiles = (nnz + 15) / 16;
    // eight waves per SIMD resident: 8,192 waves in all
    constexpr int waves = INFER_BLOCK / 64;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tiles + waves - 1) / waves, 1024 * 8 / waves));
    k_infer_bf16<<<grid, INFER_BLOCK, 0, s>>>(nnz, feat, params, rowidx, diag, m_out);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

size_t spai_probe_column_workspace_bytes(int32_t n) {
    return n < 0 ? 0 : 256 + exdot_workspace_bytes((int64_t)n) + 256;
}

int spai_probe_column(int32_t n, const double* r, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (n < 1 || !r || !out) return PBCG_ERR_INVALID;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < spai_probe_column_workspace_bytes(n)) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    double* nrm2 = (double*)ws;
    const int rc = exdot((int64_t)n, r, r, nrm2, (char*)ws + 256, ws_bytes - 256, stream);
    if (rc != PBCG_OK) return rc;
    k_probe_column<<<grid_for(n), BLOCK, 0, s>>>(n, r, nrm2, out);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int spai_probe_product(const pbcg_csr* A, const float* V, int32_t k, float* U, void* stream) {
    if (!csr_f64_ok(A) || !V || !U || k < 1) return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    k_probe_product<<<(A->n + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(A->n, k, A->row_ptr, A->col_idx,
                                                                  (const double*)A->val, V, U);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int spai_loss_grad(const pbcg_csr* A, const float* feat, const int32_t* rowidx, const double* diag,
                   const float* params, const float* V, const float* U, int32_t k, float* m_tmp, float* loss,
                   float* grad, void* ws, size_t ws_bytes, void* stream) {
    if (!csr_f64_ok(A) || !feat || !rowidx || !diag || !params || !V || !U || k < 1 || !m_tmp || !loss || !grad)
        return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < spai_workspace_bytes(A->n, A->nnz, k) || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs w = carve(ws, A->n, A->nnz, k);
    const int n = A->n;
    const int64_t nnz = A->nnz;
    const float scale_loss = 1.0f / ((float)k * (float)n);
    const float scale_grad = 2.0f / ((float)k * (float)n);
    k_forward<<<grid_for(nnz), BLOCK, 0, s>>>(nnz, feat, params, rowidx, diag, nullptr, m_tmp);
    const int nb = (n + BLOCK - 1) / BLOCK;
    k_residual<<<nb, BLOCK, 0, s>>>(n, k, A->row_ptr, A->col_idx, m_tmp, U, V, w.R, w.part);
    k_loss<<<1, 64, 0, s>>>(nb, w.part, scale_loss, loss);
    k_backward<<<grid_for(nnz), BLOCK, 0, s>>>(n, nnz, k, feat, params, rowidx, A->col_idx, diag, w.R, U,
                                                scale_grad, w.act);
    k_grad_partial<<<GRAD_BLOCKS, BLOCK, 0, s>>>(nnz, feat, w.act, w.gpart);
    k_grad_sum<<<(NPARAM + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(GRAD_BLOCKS, w.gpart, grad);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int spai_adam(float* params, float* m, float* v, const float* grad, int32_t t, float lr, float b1, float b2,
              float eps, void* stream) {
    if (!params || !m || !v || !grad || t < 1) return PBCG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    k_adam<<<(NPARAM + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(params, m, v, grad, t, lr, b1, b2, eps);
    HIPCHK(hipGetLastError());
    return PBCG_OK;
}

int spai_train_step(const pbcg_csr* A, const float* feat, const int32_t* rowidx, const double* diag,
                    const float* V, const float* U, int32_t k, float* params, float* adam_m, float* adam_v,
                    int32_t t, const float* hyper, float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (!csr_f64_ok(A) || !adam_m || !adam_v || !hyper || t < 1) return PBCG_ERR_INVALID;
    if (!ws || ws_bytes < spai_workspace_bytes(A->n, A->nnz, k) || ((uintptr_t)ws & 255)) return PBCG_ERR_WORKSPACE;
    SpaiWs w = carve(ws, A->n, A->nnz, k);
    int rc = spai_loss_grad(A, feat, rowidx, diag, params, V, U, k, w.mstep, loss, w.gstep, ws, ws_bytes, stream);
    if (rc != PBCG_OK) return rc;
    return spai_adam(params, adam_m, adam_v, w.gstep, t, hyper[0], hyper[1], hyper[2], hyper[3], stream);
}

}  // extern "C"
