/*
 * doch_oracle.h -- plain, slow, single-threaded FP64 CPU oracle for the DOCH
 * iteration (arXiv 2509.01928).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper; it is not part of the product.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Conventions
 *   - Matrices are symmetric with zero diagonal.  Sparse ones are CSR with
 *     int64 row offsets, int32 column indices (ascending within a row) and
 *     double values.  Dense ones are row-major n x n doubles.
 *   - A field h is handled by the caller building the (n+1)-spin matrix of
 *     Supp. Note 1 (eq:zero_field_ising) explicitly, see ref_augment_field.
 *   - Every floating-point quantity is double; sums run in ascending index
 *     order from 0.0.
 */
#ifndef DOCH_ORACLE_H
#define DOCH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Supp. Note 1, eq:zero_field_ising: build Jhat = [[J, h], [h^T, 0]] in CSR.
 * Outputs hold n+2 offsets, nnz+2n entries (caller-allocated). */
void ref_augment_field(int64_t n, const int64_t* rp, const int32_t* col,
                       const double* val, const double* h,
                       int64_t* rp_out, int32_t* col_out, double* val_out);

/* z = J x (CSR).  Row sums in stored (ascending column) order. */
void ref_matvec_csr(int64_t n, const int64_t* rp, const int32_t* col,
                    const double* val, const double* x, double* z);
/* z = J x (dense, row-major). */
void ref_matvec_dense(int64_t n, const double* J, const double* x, double* z);

/* eq:Hamilton: H(x) = beta/4 sum x^4 - alpha/2 sum x^2 - 1/2 x^T J x. */
double ref_hamiltonian_csr(int64_t n, const int64_t* rp, const int32_t* col,
                           const double* val, const double* x,
                           double alpha, double beta);
double ref_hamiltonian_dense(int64_t n, const double* J, const double* x,
                             double alpha, double beta);

/* DOCH (Alg. 1) with the map T of eq:FPE and the stopping rule of Remark S2.
 *   x0[n]     start vector; x_out[n] receives x^(iters_done)
 *   H_log[k]  = H(x^(k)), r_log[k] = |x^(k+1)-x^(k)|_2 / |x^(k)|_2
 *             (both length >= iters; either may be NULL)
 *   eps > 0   stop after the first k with r_log[k] < eps; eps = 0 runs iters.
 * Returns the number of iterations performed. */
int64_t ref_doch_csr(int64_t n, const int64_t* rp, const int32_t* col,
                     const double* val, const double* x0, double alpha,
                     double beta, int64_t iters, double eps, double* x_out,
                     double* H_log, double* r_log);
int64_t ref_doch_dense(int64_t n, const double* J, const double* x0,
                       double alpha, double beta, int64_t iters, double eps,
                       double* x_out, double* H_log, double* r_log);

/* ADOCH (Alg. 2, eq:BBscheme): Nesterov extrapolation accepted when
 * H(y^(k)) <= max{H(x^(j)) : max(0,k-q) <= j <= k}.  accept_log[k] = 1 if
 * y^(k) was taken (may be NULL).  Hy_log[k] = H(y^(k)) and Hmax_log[k] = the
 * window maximum it was compared with (either may be NULL), so a caller can
 * tell a clear decision from a tie within rounding.  Same logs as
 * ref_doch_csr otherwise. */
int64_t ref_adoch_csr(int64_t n, const int64_t* rp, const int32_t* col,
                      const double* val, const double* x0, double alpha,
                      double beta, int64_t iters, int32_t q, double eps,
                      double* x_out, double* H_log, double* r_log,
                      int8_t* accept_log, double* Hy_log, double* Hmax_log);

/* Alg. 1 return line: s_i = sign(x_i) with sign(0) = +1. */
void ref_sign(int64_t n, const double* x, int8_t* s);

/* eq:IsingModel: E(s) = -1/2 sum_ij J_ij s_i s_j - sum_i h_i s_i (h may be NULL). */
double ref_energy_csr_f64(int64_t n, const int64_t* rp, const int32_t* col,
                          const double* val, const double* h, const int8_t* s);
double ref_energy_dense_f64(int64_t n, const double* J, const double* h,
                            const int8_t* s);
/* Exact coupling energy -1/2 s^T J s for integer-valued J (int64 arithmetic).
 * Returns 0 on success, -1 if a value is not an integer in int32 range,
 * -2 if s^T J s is odd (impossible for a symmetric zero-diagonal J). */
int ref_energy_csr_i64(int64_t n, const int64_t* rp, const int32_t* col,
                       const double* val, const int8_t* s, int64_t* E_out);

/* Exhaustive minimum of eq:IsingModel over all 2^n spin vectors (n <= 26),
 * dense J, optional h.  s_best receives a minimiser. */
double ref_bruteforce_dense(int64_t n, const double* J, const double* h,
                            int8_t* s_best);

/* Parameter setting, eq:alphabeta / eq:estimate_eig_J / Supp. Note 6. */
/* max_i sum_{j != i} |J_ij| */
double ref_offdiag_rowsum_max(int64_t n, const int64_t* rp, const int32_t* col,
                              const double* val);
/* 2 <J> sqrt(n) with <J>^2 the off-diagonal sample variance. */
double ref_wigner_lambda(int64_t n, const int64_t* rp, const int32_t* col,
                         const double* val);
/* lambda_max(-J) by power iteration on c I - J, c = max_i sum_j |J_ij|.
 * v0[n] is the (unnormalised) start vector.  Stops when the Rayleigh quotient
 * changes by less than tol (relative) or after maxit iterations. */
double ref_power_lambda_max_neg(int64_t n, const int64_t* rp,
                                const int32_t* col, const double* val,
                                const double* v0, double tol, int64_t maxit,
                                int64_t* iters_out);

#ifdef __cplusplus
}
#endif
#endif
