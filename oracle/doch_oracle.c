/*
 * doch_oracle.c -- plain FP64 single-threaded CPU oracle of the DOCH hot path
 * (arXiv 2509.01928).  TEST INFRASTRUCTURE ONLY: loaded by the test suite,
 * the smoke check and the benchmark's CPU-baseline leg, never by the product.
 *
 * Every routine follows the paper's definitions as written, with no blocking,
 * fusion or reordering: sums run from 0.0 in ascending index order, the
 * update is evaluated as ((z_i + alpha*x_i) / beta) followed by the real cube
 * root, and the iteration is Jacobi (all coordinates from the old vector).
 *
 * Built with -O2 -ffp-contract=off and without fast-math, so each + and *
 * is one IEEE double operation.
 */
#include "doch_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- utils */

static double* dalloc(int64_t n) {
    return (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
}

/* ------------------------------------------- Supp. Note 1: homogeneous model */

void ref_augment_field(int64_t n, const int64_t* rp, const int32_t* col,
                       const double* val, const double* h,
                       int64_t* rp_out, int32_t* col_out, double* val_out) {
    /* Jhat = [[J, h], [h^T, 0]]: every row i < n gains column n with value
     * h_i (the largest column, so rows stay sorted); row n holds h^T. */
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        rp_out[i] = w;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            col_out[w] = col[e];
            val_out[w] = val[e];
            ++w;
        }
        col_out[w] = (int32_t)n;
        val_out[w] = h[i];
        ++w;
    }
    rp_out[n] = w;
    for (int64_t j = 0; j < n; ++j) {
        col_out[w] = (int32_t)j;
        val_out[w] = h[j];
        ++w;
    }
    rp_out[n + 1] = w;
}

/* ------------------------------------------------------------- matvecs */

void ref_matvec_csr(int64_t n, const int64_t* rp, const int32_t* col,
                    const double* val, const double* x, double* z) {
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc = acc + val[e] * x[col[e]];
        z[i] = acc;
    }
}

void ref_matvec_dense(int64_t n, const double* J, const double* x, double* z) {
    for (int64_t i = 0; i < n; ++i) {
        const double* row = J + i * n;
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc = acc + row[j] * x[j];
        z[i] = acc;
    }
}

/* ------------------------------------------------- eq:Hamilton, given z = Jx */

static double hamiltonian_from_z(int64_t n, const double* x, const double* z,
                                 double alpha, double beta) {
    double s4 = 0.0, s2 = 0.0, sxz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double x2 = x[i] * x[i];
        s4 = s4 + x2 * x2;
        s2 = s2 + x2;
        sxz = sxz + x[i] * z[i];
    }
    return (beta / 4.0) * s4 - (alpha / 2.0) * s2 - 0.5 * sxz;
}

double ref_hamiltonian_csr(int64_t n, const int64_t* rp, const int32_t* col,
                           const double* val, const double* x,
                           double alpha, double beta) {
    double* z = dalloc(n);
    ref_matvec_csr(n, rp, col, val, x, z);
    double H = hamiltonian_from_z(n, x, z, alpha, beta);
    free(z);
    return H;
}

double ref_hamiltonian_dense(int64_t n, const double* J, const double* x,
                             double alpha, double beta) {
    double* z = dalloc(n);
    ref_matvec_dense(n, J, x, z);
    double H = hamiltonian_from_z(n, x, z, alpha, beta);
    free(z);
    return H;
}

/* ------------------------------------------------------ eq:FPE, the map T */

/* The real cube root of eq:FPE's phi.  It is taken in x87 extended
 * precision and rounded once to double, which is correctly rounded except
 * for rare double-rounding ties (the C library's double cbrt is off by up to
 * 3 ulp on this platform). */
static double real_cbrt(double y) { return (double)cbrtl((long double)y); }

/* x_new = T(x) = cbrt((J + alpha I) x / beta), given z = J x. */
static void apply_T(int64_t n, const double* x, const double* z, double alpha,
                    double beta, double* x_new) {
    for (int64_t i = 0; i < n; ++i) {
        double y = (z[i] + alpha * x[i]) / beta;
        x_new[i] = real_cbrt(y);
    }
}

/* Remark S2: r = |x_new - x|_2 / |x|_2; r = 0 when x = 0 (then T(x) = 0). */
static double rel_step(int64_t n, const double* x, const double* x_new) {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = x_new[i] - x[i];
        num = num + d * d;
        den = den + x[i] * x[i];
    }
    if (den == 0.0) return 0.0;
    return sqrt(num) / sqrt(den);
}

/* ------------------------------------------------------------ Alg. 1 DOCH */

typedef void (*matvec_fn)(const void* A, const double* x, double* z);

typedef struct { int64_t n; const int64_t* rp; const int32_t* col; const double* val; } csr_op;
typedef struct { int64_t n; const double* J; } dense_op;

static void csr_apply(const void* A, const double* x, double* z) {
    const csr_op* a = (const csr_op*)A;
    ref_matvec_csr(a->n, a->rp, a->col, a->val, x, z);
}
static void dense_apply(const void* A, const double* x, double* z) {
    const dense_op* a = (const dense_op*)A;
    ref_matvec_dense(a->n, a->J, x, z);
}

static int64_t doch_generic(int64_t n, matvec_fn mv, const void* A,
                            const double* x0, double alpha, double beta,
                            int64_t iters, double eps, double* x_out,
                            double* H_log, double* r_log) {
    double* x = dalloc(n);
    double* xn = dalloc(n);
    double* z = dalloc(n);
    memcpy(x, x0, (size_t)n * sizeof(double));
    int64_t k = 0;
    for (; k < iters; ++k) {
        mv(A, x, z);                                   /* z = J x^(k)      */
        if (H_log) H_log[k] = hamiltonian_from_z(n, x, z, alpha, beta);
        apply_T(n, x, z, alpha, beta, xn);             /* x^(k+1) = T(x^(k)) */
        double r = rel_step(n, x, xn);
        if (r_log) r_log[k] = r;
        double* t = x; x = xn; xn = t;
        if (eps > 0.0 && r < eps) { ++k; break; }
    }
    memcpy(x_out, x, (size_t)n * sizeof(double));
    free(x); free(xn); free(z);
    return k;
}

int64_t ref_doch_csr(int64_t n, const int64_t* rp, const int32_t* col,
                     const double* val, const double* x0, double alpha,
                     double beta, int64_t iters, double eps, double* x_out,
                     double* H_log, double* r_log) {
    csr_op a = {n, rp, col, val};
    return doch_generic(n, csr_apply, &a, x0, alpha, beta, iters, eps, x_out,
                        H_log, r_log);
}

int64_t ref_doch_dense(int64_t n, const double* J, const double* x0,
                       double alpha, double beta, int64_t iters, double eps,
                       double* x_out, double* H_log, double* r_log) {
    dense_op a = {n, J};
    return doch_generic(n, dense_apply, &a, x0, alpha, beta, iters, eps, x_out,
                        H_log, r_log);
}

/* ----------------------------------------------------------- Alg. 2 ADOCH */

int64_t ref_adoch_csr(int64_t n, const int64_t* rp, const int32_t* col,
                      const double* val, const double* x0, double alpha,
                      double beta, int64_t iters, int32_t q, double eps,
                      double* x_out, double* H_log, double* r_log,
                      int8_t* accept_log, double* Hy_log, double* Hmax_log) {
    double* x = dalloc(n);      /* x^(k)   */
    double* xp = dalloc(n);     /* x^(k-1) */
    double* y = dalloc(n);
    double* xn = dalloc(n);
    double* z = dalloc(n);
    double* Hx = dalloc(iters + 1);   /* H(x^(j)) for the look-back window */
    memcpy(x, x0, (size_t)n * sizeof(double));
    memcpy(xp, x0, (size_t)n * sizeof(double));
    double t = 1.0;                   /* t_0 */
    int64_t k = 0;
    for (; k < iters; ++k) {
        double t_next = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        if (k >= 1) {
            double c = (t - 1.0) / t_next;
            for (int64_t i = 0; i < n; ++i) y[i] = x[i] + c * (x[i] - xp[i]);
        } else {
            memcpy(y, x, (size_t)n * sizeof(double));   /* y^(0) = x^(0) */
        }
        ref_matvec_csr(n, rp, col, val, x, z);
        Hx[k] = hamiltonian_from_z(n, x, z, alpha, beta);
        if (H_log) H_log[k] = Hx[k];
        double Hmax = Hx[k];
        int64_t j0 = k - q > 0 ? k - q : 0;
        for (int64_t j = j0; j <= k; ++j) if (Hx[j] > Hmax) Hmax = Hx[j];
        double* v;
        ref_matvec_csr(n, rp, col, val, y, z);
        double Hy = hamiltonian_from_z(n, y, z, alpha, beta);
        int accept = (Hy <= Hmax);
        if (Hy_log) Hy_log[k] = Hy;
        if (Hmax_log) Hmax_log[k] = Hmax;
        if (accept) {
            v = y;                                        /* z = J y  */
        } else {
            v = x;
            ref_matvec_csr(n, rp, col, val, x, z);        /* z = J x  */
        }
        if (accept_log) accept_log[k] = (int8_t)accept;
        apply_T(n, v, z, alpha, beta, xn);                /* x^(k+1) = T(v^(k)) */
        double r = rel_step(n, x, xn);
        if (r_log) r_log[k] = r;
        /* rotate: x^(k-1) <- x^(k), x^(k) <- x^(k+1) */
        double* tmp = xp; xp = x; x = xn; xn = tmp;
        t = t_next;
        if (eps > 0.0 && r < eps) { ++k; break; }
    }
    memcpy(x_out, x, (size_t)n * sizeof(double));
    free(x); free(xp); free(y); free(xn); free(z); free(Hx);
    return k;
}

/* ------------------------------------------------------- rounding, energy */

void ref_sign(int64_t n, const double* x, int8_t* s) {
    for (int64_t i = 0; i < n; ++i) s[i] = (x[i] >= 0.0) ? (int8_t)1 : (int8_t)-1;
}

double ref_energy_csr_f64(int64_t n, const int64_t* rp, const int32_t* col,
                          const double* val, const double* h, const int8_t* s) {
    double eJ = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc = acc + val[e] * (double)s[col[e]];
        eJ = eJ + (double)s[i] * acc;
    }
    double eh = 0.0;
    if (h) for (int64_t i = 0; i < n; ++i) eh = eh + h[i] * (double)s[i];
    return -0.5 * eJ - eh;
}

double ref_energy_dense_f64(int64_t n, const double* J, const double* h,
                            const int8_t* s) {
    double eJ = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc = acc + J[i * n + j] * (double)s[j];
        eJ = eJ + (double)s[i] * acc;
    }
    double eh = 0.0;
    if (h) for (int64_t i = 0; i < n; ++i) eh = eh + h[i] * (double)s[i];
    return -0.5 * eJ - eh;
}

int ref_energy_csr_i64(int64_t n, const int64_t* rp, const int32_t* col,
                       const double* val, const int8_t* s, int64_t* E_out) {
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t acc = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            double v = val[e];
            if (v != floor(v) || fabs(v) > 2147483647.0) return -1;
            acc += (int64_t)v * (int64_t)s[col[e]];
        }
        total += (int64_t)s[i] * acc;
    }
    if (total % 2 != 0) return -2;
    *E_out = -(total / 2);
    return 0;
}

/* Exhaustive search in Gray-code order.  Flipping spin i changes
 * E by 2 s_i (sum_j J_ij s_j + h_i) (s before the flip); the local fields
 * f_k = sum_j J_kj s_j + h_k are updated after every flip. */
double ref_bruteforce_dense(int64_t n, const double* J, const double* h,
                            int8_t* s_best) {
    int8_t* s = (int8_t*)malloc((size_t)n);
    double* f = dalloc(n);
    for (int64_t i = 0; i < n; ++i) s[i] = 1;
    for (int64_t k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc = acc + J[k * n + j];
        f[k] = acc + (h ? h[k] : 0.0);
    }
    double E = ref_energy_dense_f64(n, J, h, s);
    double best = E;
    memcpy(s_best, s, (size_t)n);
    uint64_t states = (uint64_t)1 << n;
    for (uint64_t t = 1; t < states; ++t) {
        int64_t i = (int64_t)__builtin_ctzll(t);
        double si = (double)s[i];
        E = E + 2.0 * si * f[i];
        for (int64_t k = 0; k < n; ++k) f[k] = f[k] - 2.0 * J[k * n + i] * si;
        s[i] = (int8_t)(-s[i]);
        if (E < best) { best = E; memcpy(s_best, s, (size_t)n); }
    }
    free(s); free(f);
    /* report the exact energy of the minimiser, not the running sum */
    return ref_energy_dense_f64(n, J, h, s_best);
}

/* ------------------------------------------------------ parameter setting */

double ref_offdiag_rowsum_max(int64_t n, const int64_t* rp, const int32_t* col,
                              const double* val) {
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] != i) acc = acc + fabs(val[e]);
        if (acc > best) best = acc;
    }
    return best;
}

double ref_wigner_lambda(int64_t n, const int64_t* rp, const int32_t* col,
                         const double* val) {
    /* eq:estimate_eig_J over the n(n-1) off-diagonal entries (zeros included):
     * Jbar = S1/(n(n-1)), <J>^2 = sum_{i!=j} (J_ij - Jbar)^2 / (n(n-1)). */
    double m = (double)n * (double)(n - 1);
    double s1 = 0.0;
    int64_t stored = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] != i) { s1 = s1 + val[e]; ++stored; }
    double jbar = s1 / m;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] != i) { double d = val[e] - jbar; ss = ss + d * d; }
    /* the off-diagonal entries that are not stored are zeros */
    ss = ss + (m - (double)stored) * jbar * jbar;
    double var = ss / m;
    return 2.0 * sqrt(var) * sqrt((double)n);
}

double ref_power_lambda_max_neg(int64_t n, const int64_t* rp,
                                const int32_t* col, const double* val,
                                const double* v0, double tol, int64_t maxit,
                                int64_t* iters_out) {
    /* c = max_i sum_j |J_ij| bounds every |eigenvalue|, so c I - J is PSD
     * and its dominant eigenvalue is c - lambda_min(J) = c + lambda_max(-J). */
    double c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc = acc + fabs(val[e]);
        if (acc > c) c = acc;
    }
    double* v = dalloc(n);
    double* w = dalloc(n);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) nrm = nrm + v0[i] * v0[i];
    nrm = sqrt(nrm);
    for (int64_t i = 0; i < n; ++i) v[i] = v0[i] / nrm;
    double mu = 0.0, mu_prev = 0.0;
    int64_t it = 0;
    for (; it < maxit; ++it) {
        ref_matvec_csr(n, rp, col, val, v, w);
        for (int64_t i = 0; i < n; ++i) w[i] = c * v[i] - w[i];   /* (cI - J) v */
        double rq = 0.0, ww = 0.0;
        for (int64_t i = 0; i < n; ++i) { rq = rq + v[i] * w[i]; ww = ww + w[i] * w[i]; }
        mu = rq;                                                  /* Rayleigh quotient */
        ww = sqrt(ww);
        if (ww == 0.0) break;
        for (int64_t i = 0; i < n; ++i) v[i] = w[i] / ww;
        if (it > 0 && fabs(mu - mu_prev) <= tol * fabs(mu)) { ++it; break; }
        mu_prev = mu;
    }
    if (iters_out) *iters_out = it;
    free(v); free(w);
    return mu - c;
}
