/*
 * CPU oracle, tier 2 -- TEST INFRASTRUCTURE ONLY (plain C + OpenMP).
 *
 * The same definitions as the Python tier (oracle/exact.py, oracle/spmv.py,
 * oracle/solvers.py), written independently in C so that large inputs can be
 * checked and the CPU baseline timed:
 *
 *   ora_exact_dot  RN_even(sum x_i y_i) with the sum formed exactly
 *                  (paper Section 2, the ExBLAS paragraph): every product of
 *                  doubles is an integer multiple of 2^-2148; the products are
 *                  added into a two's-complement integer of 68 x 64-bit limbs
 *                  (bit k of the integer has weight 2^(k-2148)) and the integer is
 *                  rounded once to nearest-even.
 *   ora_spmv       CSR row sums, left to right, multiply and add rounded separately.
 *   ora_pbicgstab  Algorithm 2 with the readings listed in oracle/solvers.py.
 *   ora_bicgstab   Algorithm 1.
 *
 * Built with -O2 -ffp-contract=off (no FMA contraction of the recurrences).
 * Shares no code with the HIP library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NLIMB 68            /* 4352 bits: 2^-2148 .. 2^2204 incl. carry headroom */
#define BIAS 2148

typedef struct {
    uint64_t w[NLIMB];
    int nan, pinf, ninf;
} acc_t;

static void acc_zero(acc_t* a) { memset(a, 0, sizeof(*a)); }

/* value = m * 2^e, m < 2^53 unsigned, sign separate */
static void split(double d, uint64_t* m, int* e, int* neg) {
    uint64_t bits;
    memcpy(&bits, &d, 8);
    *neg = (int)(bits >> 63);
    int be = (int)((bits >> 52) & 0x7ff);
    uint64_t f = bits & ((1ull << 52) - 1);
    if (be == 0) { *m = f; *e = -1074; }
    else { *m = f | (1ull << 52); *e = be - 1075; }
}

/* add (neg ? -1 : 1) * v * 2^pos into the limb integer, v < 2^128 */
static void acc_add_shifted(acc_t* a, unsigned __int128 v, int pos, int neg) {
    int li = pos >> 6, sh = pos & 63;
    uint64_t p0 = (uint64_t)v, p1 = (uint64_t)(v >> 64);
    uint64_t t[3];
    t[0] = p0 << sh;
    t[1] = sh ? ((p1 << sh) | (p0 >> (64 - sh))) : p1;
    t[2] = sh ? (p1 >> (64 - sh)) : 0;
    if (!neg) {
        uint64_t carry = 0;
        for (int k = 0; k < 3 || carry; ++k) {
            int j = li + k;
            if (j >= NLIMB) break;
            uint64_t add = k < 3 ? t[k] : 0;
            uint64_t s = a->w[j] + add;
            uint64_t c1 = s < add;
            uint64_t s2 = s + carry;
            uint64_t c2 = s2 < carry;
            a->w[j] = s2;
            carry = c1 | c2;
            if (k >= 2 && !carry) break;
        }
    } else {
        uint64_t borrow = 0;
        for (int k = 0; k < 3 || borrow; ++k) {
            int j = li + k;
            if (j >= NLIMB) break;
            uint64_t sub = k < 3 ? t[k] : 0;
            uint64_t old = a->w[j];
            uint64_t s = old - sub;
            uint64_t b1 = old < sub;
            uint64_t s2 = s - borrow;
            uint64_t b2 = s < borrow;
            a->w[j] = s2;
            borrow = b1 | b2;
            if (k >= 2 && !borrow) break;
        }
    }
}

static void acc_add_product(acc_t* a, double x, double y) {
    if (isnan(x) || isnan(y)) { a->nan = 1; return; }
    if (isinf(x) || isinf(y)) {
        if (x == 0.0 || y == 0.0) { a->nan = 1; return; }
        if ((x > 0) == (y > 0)) a->pinf = 1; else a->ninf = 1;
        return;
    }
    if (x == 0.0 || y == 0.0) return;
    uint64_t mx, my; int ex, ey, nx, ny;
    split(x, &mx, &ex, &nx);
    split(y, &my, &ey, &ny);
    unsigned __int128 prod = (unsigned __int128)mx * my;
    acc_add_shifted(a, prod, ex + ey + BIAS, nx ^ ny);
}

static void acc_merge(acc_t* dst, const acc_t* src) {
    uint64_t carry = 0;
    for (int j = 0; j < NLIMB; ++j) {
        uint64_t s = dst->w[j] + src->w[j];
        uint64_t c1 = s < src->w[j];
        uint64_t s2 = s + carry;
        uint64_t c2 = s2 < carry;
        dst->w[j] = s2;
        carry = c1 | c2;
    }
    dst->nan |= src->nan; dst->pinf |= src->pinf; dst->ninf |= src->ninf;
}

/* bit k of the magnitude integer */
static int getbit(const uint64_t* w, int k) {
    if (k < 0) return 0;
    return (int)((w[k >> 6] >> (k & 63)) & 1);
}

static int any_below(const uint64_t* w, int k) { /* any bit with index < k set */
    if (k <= 0) return 0;
    int li = k >> 6, sh = k & 63;
    for (int j = 0; j < li; ++j) if (w[j]) return 1;
    if (sh && (w[li] & ((1ull << sh) - 1))) return 1;
    return 0;
}

static double acc_round(const acc_t* a) {
    if (a->nan || (a->pinf && a->ninf)) return NAN;
    if (a->pinf) return INFINITY;
    if (a->ninf) return -INFINITY;
    uint64_t mag[NLIMB];
    int neg = (int)(a->w[NLIMB - 1] >> 63);
    if (neg) { /* two's complement negate */
        uint64_t carry = 1;
        for (int j = 0; j < NLIMB; ++j) {
            uint64_t v = ~a->w[j];
            mag[j] = v + carry;
            carry = (mag[j] < carry);
        }
    } else {
        memcpy(mag, a->w, sizeof(mag));
    }
    int top = -1;
    for (int j = NLIMB - 1; j >= 0; --j) if (mag[j]) { top = j; break; }
    if (top < 0) return 0.0;
    int msb = top * 64 + 63 - __builtin_clzll(mag[top]);
    /* exponent of the leading bit: msb - BIAS.  Normal if >= -1022. */
    int lead = msb - BIAS;
    int lsb;                      /* integer bit index of the unit in the last place */
    if (lead >= -1022) lsb = msb - 52;
    else lsb = -1074 + BIAS;       /* subnormal: fixed quantum 2^-1074 */
    uint64_t mant = 0;
    for (int k = msb; k >= lsb; --k) mant = (mant << 1) | (uint64_t)getbit(mag, k);
    int guard = getbit(mag, lsb - 1);
    int sticky = any_below(mag, lsb - 1);
    if (guard && (sticky || (mant & 1))) mant += 1;
    /* value = mant * 2^(lsb - BIAS) */
    double r;
    if (lead >= -1022) {
        int e = lsb - BIAS;
        if (mant == (1ull << 53)) { mant >>= 1; e += 1; }
        if (e + 52 > 1023) r = INFINITY;
        else r = ldexp((double)mant, e);   /* exact: mant < 2^53 */
    } else {
        r = ldexp((double)mant, -1074);    /* exact: mant <= 2^52 */
    }
    return neg ? -r : r;
}

double ora_exact_dot(const double* x, const double* y, int64_t n) {
    int nt = omp_get_max_threads();
    acc_t* parts = (acc_t*)calloc((size_t)nt, sizeof(acc_t));
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        acc_t* a = &parts[tid];
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) acc_add_product(a, x[i], y[i]);
    }
    acc_t tot;
    acc_zero(&tot);
    for (int t = 0; t < nt; ++t) acc_merge(&tot, &parts[t]);
    free(parts);
    return acc_round(&tot);
}

/* round a caller-provided scaled integer: limbs little-endian two's complement */
double ora_round_limbs(const uint64_t* limbs) {
    acc_t a;
    acc_zero(&a);
    memcpy(a.w, limbs, sizeof(a.w));
    return acc_round(&a);
}

void ora_spmv(int32_t n, const int32_t* rp, const int32_t* ci, const double* val,
              const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            double prod = val[k] * x[ci[k]];
            s = s + prod;
        }
        y[i] = s;
    }
}

enum { S_OK = 0, S_NOT_CONVERGED = 1, S_BREAKDOWN = 2, S_STAGNATED = 3, S_ERR_NONFINITE = -3 };

/* The stopping test: the first true-residual test comes when rec <= tol; after a
 * failed test the next comes 5 iterations later; a failed test below every earlier one
 * keeps its iterate (in xb); 30 failed tests in a row without a new best mean
 * stagnation. */
typedef struct { double lim, best; int stag, it_fail; double* xb; } true_test;
static int tt_due(const true_test* t, double rec, double tol, int it) {
    if (t->it_fail < 0) return rec <= tol;
    return it - t->it_fail >= 5;
}
static int tt_failed(true_test* t, double rec, double tr, int it, const double* x, int32_t n) {
    (void)rec;
    t->it_fail = it;
    if (tr < t->best) {
        t->best = tr; t->stag = 0;
        memcpy(t->xb, x, sizeof(double) * (size_t)n);
        return 0;
    }
    return ++t->stag >= 30;
}

typedef struct {
    int32_t status, iterations, true_checks, pad;
    double true_relres, rec_relres;
} ora_info;

static double true_relres(int32_t n, const int32_t* rp, const int32_t* ci, const double* val,
                          const double* b, const double* x, double normb, double* tmp) {
    ora_spmv(n, rp, ci, val, x, tmp);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) tmp[i] = b[i] - tmp[i];
    return sqrt(ora_exact_dot(tmp, tmp, n)) / normb;
}

#define ALLOCV(name) double* name = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1))

/* Algorithm 2; x holds x0 on entry and the final iterate on exit.
 * hist (optional, length max_iter) receives the recursive relative residuals. */
int ora_pbicgstab(int32_t n, const int32_t* rp, const int32_t* ci, const double* val,
                  const double* b, double* x, double tol, int32_t max_iter,
                  ora_info* info, double* hist) {
    ALLOCV(r); ALLOCV(rh); ALLOCV(w); ALLOCV(t); ALLOCV(p); ALLOCV(s); ALLOCV(z);
    ALLOCV(q); ALLOCV(y); ALLOCV(v); ALLOCV(tmp); ALLOCV(xbest);
    int status = S_NOT_CONVERGED, iters = 0, checks = 0;
    double rec = NAN, tr = NAN;
    double nb2 = ora_exact_dot(b, b, n);
    if (!isfinite(nb2)) { status = S_ERR_NONFINITE; goto done; }
    double normb = sqrt(nb2);
    if (normb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        status = S_OK; rec = tr = 0.0; goto done;
    }
    ora_spmv(n, rp, ci, val, x, tmp);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { r[i] = b[i] - tmp[i]; rh[i] = r[i]; }
    ora_spmv(n, rp, ci, val, r, w);
    ora_spmv(n, rp, ci, val, w, t);
    double rho = ora_exact_dot(rh, r, n);
    double rw = ora_exact_dot(rh, w, n);
    rec = sqrt(ora_exact_dot(r, r, n)) / normb;
    true_test tt = {INFINITY, INFINITY, 0, -1, xbest};
    if (tt_due(&tt, rec, tol, 0)) {
        checks++;
        tr = true_relres(n, rp, ci, val, b, x, normb, tmp);
        if (tr <= tol) { status = S_OK; goto done_tr; }
        if (tt_failed(&tt, rec, tr, 0, x, n)) {
            memcpy(x, xbest, sizeof(double) * (size_t)n);
            tr = tt.best; status = S_STAGNATED; goto done_tr;
        }
    }
    if (!isfinite(rho) || !isfinite(rw)) { status = S_ERR_NONFINITE; goto done; }
    if (rw == 0.0) { status = S_BREAKDOWN; goto done; }
    double alpha = rho / rw, beta = 0.0, omega = 0.0;
    for (int32_t it = 0; it < max_iter; ++it) {
        if (it == 0) {
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i) { p[i] = r[i]; s[i] = w[i]; z[i] = t[i]; }
        } else {
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i) {
                p[i] = r[i] + beta * (p[i] - omega * s[i]);
                s[i] = w[i] + beta * (s[i] - omega * z[i]);
                z[i] = t[i] + beta * (z[i] - omega * v[i]);
            }
        }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) { q[i] = r[i] - alpha * s[i]; y[i] = w[i] - alpha * z[i]; }
        double qy = ora_exact_dot(q, y, n), yy = ora_exact_dot(y, y, n);
        double rs = ora_exact_dot(rh, s, n), rz = ora_exact_dot(rh, z, n);
        ora_spmv(n, rp, ci, val, z, v);
        if (!isfinite(qy) || !isfinite(yy) || !isfinite(rs) || !isfinite(rz)) {
            status = S_ERR_NONFINITE; iters = it; goto done;
        }
        if (yy == 0.0) {
            if (ora_exact_dot(q, q, n) == 0.0) {
#pragma omp parallel for schedule(static)
                for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
                iters = it + 1; checks++; rec = 0.0;
                tr = true_relres(n, rp, ci, val, b, x, normb, tmp);
                status = tr <= tol ? S_OK : S_BREAKDOWN;
                goto done_tr;
            }
            status = S_BREAKDOWN; iters = it; goto done;
        }
        omega = qy / yy;
        if (omega == 0.0) { status = S_BREAKDOWN; iters = it; goto done; }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            x[i] = (x[i] + alpha * p[i]) + omega * q[i];
            r[i] = q[i] - omega * y[i];
            w[i] = y[i] - omega * (t[i] - alpha * v[i]);
        }
        ora_spmv(n, rp, ci, val, w, t);
        double rho_new = ora_exact_dot(rh, r, n);
        rw = ora_exact_dot(rh, w, n);
        double rr = ora_exact_dot(r, r, n);
        rec = sqrt(rr) / normb;
        if (hist) hist[it] = rec;
        iters = it + 1;
        beta = ((alpha / omega) * rho_new) / rho;
        double den = (rw + beta * rs) - (beta * omega) * rz;
        double alpha_new = den != 0.0 ? rho_new / den : NAN;
        if (tt_due(&tt, rec, tol, it + 1)) {
            checks++;
            tr = true_relres(n, rp, ci, val, b, x, normb, tmp);
            if (tr <= tol) { status = S_OK; goto done_tr; }
            if (tt_failed(&tt, rec, tr, it + 1, x, n)) {
                memcpy(x, xbest, sizeof(double) * (size_t)n);
                tr = tt.best; status = S_STAGNATED; goto done_tr;
            }
        }
        if (!isfinite(rho_new) || !isfinite(rw) || !isfinite(rr) || !isfinite(beta) ||
            (den != 0.0 && !isfinite(alpha_new))) { status = S_ERR_NONFINITE; goto done; }
        if (rho_new == 0.0 || den == 0.0) { status = S_BREAKDOWN; goto done; }
        alpha = alpha_new; rho = rho_new;
    }
    status = S_NOT_CONVERGED;
done:
    tr = (status == S_ERR_NONFINITE && !isfinite(nb2)) ? NAN
         : true_relres(n, rp, ci, val, b, x, sqrt(nb2), tmp);
done_tr:
    if (info) {
        info->status = status; info->iterations = iters; info->true_checks = checks;
        info->true_relres = tr; info->rec_relres = rec;
    }
    free(r); free(rh); free(w); free(t); free(p); free(s); free(z); free(q); free(y); free(v); free(tmp); free(xbest);
    return status;
}

/* Algorithm 1 (BiCGStab), same conventions. */
int ora_bicgstab(int32_t n, const int32_t* rp, const int32_t* ci, const double* val,
                 const double* b, double* x, double tol, int32_t max_iter,
                 ora_info* info, double* hist) {
    ALLOCV(r); ALLOCV(rh); ALLOCV(p); ALLOCV(s); ALLOCV(q); ALLOCV(y); ALLOCV(tmp); ALLOCV(xbest);
    int status = S_NOT_CONVERGED, iters = 0, checks = 0;
    double rec = NAN, tr = NAN;
    double nb2 = ora_exact_dot(b, b, n);
    if (!isfinite(nb2)) { status = S_ERR_NONFINITE; goto done; }
    double normb = sqrt(nb2);
    if (normb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        status = S_OK; rec = tr = 0.0; goto done_tr;
    }
    ora_spmv(n, rp, ci, val, x, tmp);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { r[i] = b[i] - tmp[i]; rh[i] = r[i]; p[i] = r[i]; }
    double rho = ora_exact_dot(rh, r, n);
    rec = sqrt(ora_exact_dot(r, r, n)) / normb;
    true_test tt = {INFINITY, INFINITY, 0, -1, xbest};
    if (tt_due(&tt, rec, tol, 0)) {
        checks++;
        tr = true_relres(n, rp, ci, val, b, x, normb, tmp);
        if (tr <= tol) { status = S_OK; goto done_tr; }
        if (tt_failed(&tt, rec, tr, 0, x, n)) {
            memcpy(x, xbest, sizeof(double) * (size_t)n);
            tr = tt.best; status = S_STAGNATED; goto done_tr;
        }
    }
    if (!isfinite(rho)) { status = S_ERR_NONFINITE; goto done; }
    for (int32_t it = 0; it < max_iter; ++it) {
        ora_spmv(n, rp, ci, val, p, s);
        double rs = ora_exact_dot(rh, s, n);
        if (!isfinite(rs)) { status = S_ERR_NONFINITE; iters = it; goto done; }
        if (rs == 0.0 || rho == 0.0) { status = S_BREAKDOWN; iters = it; goto done; }
        double alpha = rho / rs;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) q[i] = r[i] - alpha * s[i];
        ora_spmv(n, rp, ci, val, q, y);
        double qy = ora_exact_dot(q, y, n), yy = ora_exact_dot(y, y, n);
        if (!isfinite(qy) || !isfinite(yy)) { status = S_ERR_NONFINITE; iters = it; goto done; }
        if (yy == 0.0) {
            if (ora_exact_dot(q, q, n) == 0.0) {
#pragma omp parallel for schedule(static)
                for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
                iters = it + 1; checks++; rec = 0.0;
                tr = true_relres(n, rp, ci, val, b, x, normb, tmp);
                status = tr <= tol ? S_OK : S_BREAKDOWN;
                goto done_tr;
            }
            status = S_BREAKDOWN; iters = it; goto done;
        }
        double omega = qy / yy;
        if (omega == 0.0) { status = S_BREAKDOWN; iters = it; goto done; }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            x[i] = (x[i] + alpha * p[i]) + omega * q[i];
            r[i] = q[i] - omega * y[i];
        }
        double rho_new = ora_exact_dot(rh, r, n);
        double rr = ora_exact_dot(r, r, n);
        rec = sqrt(rr) / normb;
        if (hist) hist[it] = rec;
        iters = it + 1;
        double beta = ((alpha / omega) * rho_new) / rho;
        if (tt_due(&tt, rec, tol, it + 1)) {
            checks++;
            tr = true_relres(n, rp, ci, val, b, x, normb, tmp);
            if (tr <= tol) { status = S_OK; goto done_tr; }
            if (tt_failed(&tt, rec, tr, it + 1, x, n)) {
                memcpy(x, xbest, sizeof(double) * (size_t)n);
                tr = tt.best; status = S_STAGNATED; goto done_tr;
            }
        }
        if (!isfinite(rho_new) || !isfinite(rr) || !isfinite(beta)) { status = S_ERR_NONFINITE; goto done; }
        if (rho_new == 0.0) { status = S_BREAKDOWN; goto done; }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * s[i]);
        rho = rho_new;
    }
    status = S_NOT_CONVERGED;
done:
    tr = (status == S_ERR_NONFINITE && !isfinite(nb2)) ? NAN
         : true_relres(n, rp, ci, val, b, x, sqrt(nb2), tmp);
done_tr:
    if (info) {
        info->status = status; info->iterations = iters; info->true_checks = checks;
        info->true_relres = tr; info->rec_relres = rec;
    }
    free(r); free(rh); free(p); free(s); free(q); free(y); free(tmp); free(xbest);
    return status;
}

int ora_num_threads(void) { return omp_get_max_threads(); }
void ora_set_threads(int nt) { if (nt > 0) omp_set_num_threads(nt); }
