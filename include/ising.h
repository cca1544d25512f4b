/*
 * ising.h -- C ABI of the MI355X (gfx950) DOCH library.
 *
 * DOCH (arXiv 2509.01928, Methods, Alg. 1) minimises the Hamiltonian
 *   H(x) = beta/4 sum_i x_i^4 - alpha/2 sum_i x_i^2 - 1/2 x^T J x   (eq:Hamilton)
 * by the fixed-point map
 *   x^(k+1) = T(x^(k)),  T(x) = cbrt((J + alpha I) x / beta)          (eq:FPE)
 * and returns s = sign(x^(N)).  The Ising energy of eq:IsingModel,
 *   E(s) = -1/2 sum_ij J_ij s_i s_j - sum_i h_i s_i,
 * scores the result.  A field h is handled through the homogeneous model of
 * Supp. Note 1 (eq:zero_field_ising): one extra spin t couples to spin i with
 * weight h_i, the iteration runs on n' = n + 1 variables and the answer is
 * s_i = sign(t) sign(x_i) (Prop. S1).
 *
 * Conventions for every entry point
 *   - Pointers named *_dev are device pointers on the current HIP device;
 *     pointers named *_host are host pointers.  The caller owns them all.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it asynchronously unless stated otherwise.
 *   - Every call returns an ising_status and never aborts the process.
 *     Arguments are validated before any device write, so a failed call
 *     leaves outputs untouched.  ising_last_error() gives the detail text of
 *     the last failure on the calling thread.
 *   - A context is not thread-safe: one solve at a time per context.
 *     Distinct contexts are independent.
 *   - Iterates use restart-interleaved storage: a block of R start vectors
 *     is an n' x R row-major array, element (i, r) at index i*R + r.
 *     When the problem has a field, row n holds the extra spin t.
 */
#ifndef ISING_H
#define ISING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ising_ctx ising_ctx;   /* opaque, owned by the library */

typedef enum {
    ISING_OK = 0,
    ISING_E_INVALID_ARG = 1,     /* bad size, NULL pointer, bad enum        */
    ISING_E_NONZERO_DIAG = 2,    /* J_ii != 0 (eq:IsingModel needs J_ii = 0) */
    ISING_E_NOT_SYMMETRIC = 3,   /* J != J^T (checked by ising_check_symmetric) */
    ISING_E_OUT_OF_MEMORY = 4,
    ISING_E_HIP = 5,             /* a HIP runtime call failed               */
    ISING_E_UNSUPPORTED = 6,     /* valid request the library does not serve */
    ISING_E_NONFINITE = 7        /* H or r became non-finite during a solve */
} ising_status;

typedef enum {
    ISING_F64 = 0,
    ISING_F32 = 1,
    ISING_BF16 = 2,
    ISING_FP8_E4M3 = 3,
    ISING_I32 = 4,
    ISING_I16 = 5      /* 16-bit signed integer CSR values (the 9-bit workload) */
} ising_dtype;

/* Solver parameters.  alpha and beta are the attractor parameters of
 * eq:attractor (the "potential params"); eq:alphabeta gives the recommended
 * values, see ising_default_params. */
typedef struct {
    double alpha;          /* > 0                                            */
    double beta;           /* > 0                                            */
    double eps;            /* Remark S2 tolerance on r^(k); 0 = run `iters`   */
    int32_t algo;          /* 0 = DOCH (Alg. 1); 1 = ADOCH (Alg. 2)          */
    int32_t q;             /* ADOCH look-back window (Alg. 2), >= 1          */
    int32_t x_dtype;       /* ising_dtype storing the iterate: ISING_F64 or
                              ISING_F32 (arithmetic is FP64 in both)          */
    int32_t reserved;      /* must be 0                                      */
} ising_params;

/* Per-restart result of a solve. */
typedef struct {
    int64_t iters_done;    /* iterations performed (<= iters)                */
    int32_t converged;     /* 1 if r^(k) < eps stopped the run               */
    int32_t nonfinite;     /* 1 if H or r became non-finite                  */
    double H_last;         /* H(x^(iters_done-1)), eq:Hamilton               */
    double r_last;         /* r^(iters_done-1), Remark S2                    */
} ising_stats;

/* Facts about a context. */
typedef struct {
    int64_t n;             /* spins                                          */
    int64_t n_iter;        /* n' = n + (field ? 1 : 0), length of an iterate */
    int64_t nnz;           /* stored couplings (CSR) or n*(n-1) (dense)      */
    int32_t is_dense;
    int32_t has_field;
    int32_t integer_J;     /* all couplings are integers (exact int64 energy) */
    int32_t val_dtype;     /* ising_dtype the couplings are stored in        */
    int32_t row_len;       /* CSR: d if every row holds d entries (row i
                              starts at d*i; the lane-per-row kernels then
                              do not read the offsets), else 0             */
    int32_t geometry;      /* geometry single-restart solves use (see
                              ising_set_geometry): 0..8 for CSR; -1
                              (automatic), 0 or 8 for dense; -1 for batches */
    int32_t step_val_bytes; /* bytes per coupling value the lane-per-row
                              CSR step (geometries 3, 4) streams: 1 when
                              every value is an integer in [-128, 127] (the
                              library then keeps an exact 8-bit copy beside
                              the values, nnz more bytes of device memory;
                              the ADOCH product and the eta sweep on rows of
                              4 entries read it too), else the size of
                              val_dtype; 8 for dense                       */
    int32_t step_col_bytes; /* bytes per column index that step streams: 2
                              when every row holds 4 entries, the 8-bit
                              value copy is kept and every column lies
                              within 32767 of its row modulo n (the library
                              then keeps each entry's offset col - i as 16
                              bits, 2 nnz more bytes; the ADOCH product
                              reads it too); else 4; 0 for dense           */
} ising_info;

/* ---------------------------------------------------------------- create
 * Copy a symmetric coupling matrix J (J_ii = 0) and an optional field h into
 * library-owned device memory.  Synchronises `stream` before returning; the
 * caller may free its buffers afterwards.
 *
 * ising_create_csr: CSR of the full matrix (both triangles), as used for the
 * sparse instances of Supp. Note 9.
 *   n            spins, 1 <= n < 2^31 - 1
 *   nnz          stored entries, 0 <= nnz < 2^31
 *   row_ptr_dev  int32[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_dev      int32[nnz], 0 <= col < n, ascending within each row
 *   val_dev      nnz values of type vt: ISING_F32, ISING_F64, or ISING_I16
 *                for integer couplings (6 bytes per stored entry with the
 *                index; the 9-bit workload of Supp. Alg. S5)
 *   h_dev        NULL (no field) or n values of type ht (ISING_F32 / F64)
 * Errors: ISING_E_INVALID_ARG for a malformed CSR (checked on the device),
 * ISING_E_NONZERO_DIAG if a stored diagonal entry is nonzero.
 * Symmetry is not checked here (see ising_check_symmetric). */
ising_status ising_create_csr(int64_t n, int64_t nnz, const int32_t* row_ptr_dev,
                              const int32_t* col_dev, const void* val_dev,
                              int32_t vt, const void* h_dev, int32_t ht,
                              void* stream, ising_ctx** out);

/* ising_create_dense: row-major dense J with leading dimension ld >= n.
 *   J_dev  n x ld values of type jt (ISING_F64)
 *   h_dev  as above.
 * Errors: ISING_E_INVALID_ARG, ISING_E_NONZERO_DIAG. */
ising_status ising_create_dense(int64_t n, const void* J_dev, int32_t jt, int64_t ld,
                                const void* h_dev, int32_t ht, void* stream,
                                ising_ctx** out);

/* ising_create_procedural: a dense context whose couplings are generated on
 * demand instead of stored (Supp. Note 9): kind 1 is J_ij = sin(i*j + seed)
 * with 0-based indices i, j and J_ii = 0, evaluated in FP64; the paper uses
 * seed = 100.  The seed must be an integer with |seed| + (n-1)^2 < 2^53, so
 * that every argument i*j + seed is an exact FP64 integer (the kernels step
 * the angle exactly and restart from exact arguments); other seeds give
 * ISING_E_INVALID_ARG, as do n < 2 or n > 9e7.  No field.  Every entry
 * point that takes a dense context accepts it except ising_solve_lowp.  It
 * allocates nothing until used. */
ising_status ising_create_procedural(int64_t n, int32_t kind, double seed, void* stream,
                                     ising_ctx** out);

/* Release a context and all its device memory (NULL is ignored). */
void ising_destroy(ising_ctx* ctx);

ising_status ising_get_info(const ising_ctx* ctx, ising_info* out);

/* Check J == J^T exactly on the device (CSR: every (i,j,v) has a matching
 * (j,i,v)).  Synchronous.  ISING_OK or ISING_E_NOT_SYMMETRIC. */
ising_status ising_check_symmetric(ising_ctx* ctx, void* stream);

/* ------------------------------------------------------- parameter setting
 * eq:alphabeta with Supp. Note 6, on the homogeneous matrix Jhat (n' spins):
 *   lambda = lambda_max(-Jhat): power iteration on c I - Jhat,
 *            c = max_i sum_j |Jhat_ij|, when n' < 10^4 (stops when the
 *            Rayleigh quotient changes by <= 1e-12 relative, at most 1e5
 *            iterations); otherwise Wigner's estimate 2 <Jhat> sqrt(n') with
 *            <Jhat>^2 the sample variance of the n'(n'-1) off-diagonal
 *            entries (eq:estimate_eig_J)
 *   alpha  = eta * lambda
 *   beta   = n'^(3/2) * (alpha + max_i sum_{j != i} |Jhat_ij|)
 * Fills *out (eps = 0, algo = 0, q = 5, x_dtype = ISING_F64) and writes the
 * lambda used to *lambda_out when non-NULL.  Synchronous on `stream`.
 * method: 0 = as above, 1 = always power iteration, 2 = always Wigner. */
ising_status ising_default_params(ising_ctx* ctx, double eta, int32_t method,
                                  void* stream, ising_params* out,
                                  double* lambda_out);

/* Supp. Note 6: choose eta by short probe runs.  lambda_hat and the row-sum
 * bound are estimated once as by ising_default_params (`method`); for each
 * eta_k, alpha = eta_k lambda_hat and beta follow eq:alphabeta, DOCH runs
 * `probe_iters` iterations from x0_dev (as for ising_solve with R = 1), the
 * iterate is rounded and its Ising energy (eq:IsingModel) taken.  The eta
 * with the lowest energy wins (the first one on a tie).  On a CSR or a
 * procedural context the probes run eight at a time as restarts of one pass
 * over the couplings (a lone remaining probe on the single-restart path);
 * every probe's iterates, and so its energy, are those of a single-restart
 * solve with its parameters.  A stored dense context runs them one after
 * another.
 *   count          1..64 candidates, etas_host[k] in (0, 2]
 *   probe_iters    1..1000 (the paper uses 5-10, 1-3 for ultra-large graphs)
 *   best_out       the winner's ising_params (eps 0, algo 0, q 5, FP64 iterate)
 *   best_eta_out   NULL or the winning eta
 *   energies_host  NULL or count doubles: every probe's energy
 * Synchronous.  May overwrite the log of the last solve.  Errors: as
 * ising_default_params and ising_solve; ISING_E_UNSUPPORTED on a batch
 * context. */
ising_status ising_tune_eta(ising_ctx* ctx, const double* x0_dev, int32_t count,
                            const double* etas_host, int64_t probe_iters, int32_t method,
                            void* stream, ising_params* best_out, double* best_eta_out,
                            double* energies_host);

/* ------------------------------------------------------------------ solve
 * Run `iters` iterations of DOCH (Alg. 1) -- or ADOCH (Alg. 2) when
 * params->algo == 1 -- from R start vectors at once, then round.
 *   x0_dev    double[n' * R] start vectors (interleaved, see above)
 *   R         restarts, 1 <= R <= 1024
 *   iters     >= 0
 *   x_out_dev NULL or double[n' * R]: the final iterates x^(iters_done)
 *   s_out_dev NULL or int8[n * R]: spins s_i = sign(x_i) (sign(0) = +1),
 *             multiplied by sign(t) when there is a field
 *   stats_host NULL or ising_stats[R]; when given, the call synchronises
 *             `stream` and fills it.
 * Each restart stops on its own when params->eps > 0 and r^(k) < eps.
 * H(x^(k)) and r^(k) of every iteration are kept for ising_get_log.
 * Errors: ISING_E_INVALID_ARG; ISING_E_NONFINITE (only detectable when
 * stats_host is given) if H or r became non-finite -- the restart then
 * stops at that iteration. */
ising_status ising_solve(ising_ctx* ctx, const double* x0_dev, int32_t R,
                         int64_t iters, const ising_params* params,
                         double* x_out_dev, int8_t* s_out_dev,
                         ising_stats* stats_host, void* stream);

/* ADOCH (params->algo = 1, Alg. 2 with the window of eq:BBscheme) runs on
 * single CSR and dense contexts (stored or generated couplings) with R in
 * {1, 2, 4, 8} restarts together and FP64 iterates (ISING_E_UNSUPPORTED
 * otherwise); params->q >= 1 is the look-back window.  Every restart keeps
 * its own window, decisions and stopping (Remark S2 with params->eps), and
 * ising_get_log(restart) reads its H and r.  It still costs one matvec per
 * iteration: J y is formed from J x^(k) and J x^(k-1).  One restart on a
 * stored dense matrix of order <= 2048 without a field, q <= 63 and at most
 * 10^7 iterations runs resident (one cooperative launch for the whole run)
 * unless ising_set_geometry chose geometry 0; the first call with more
 * iterations than any before on the context synchronises the stream (the
 * momentum weights are uploaded once).
 * ising_get_accept_log copies, for the last ADOCH solve, whether iteration
 * first + i of restart r took the extrapolated point (1) or x^(k) (0), at
 * accept_host[i * R + r] (count * R entries).  Synchronous. */
ising_status ising_get_accept_log(ising_ctx* ctx, int64_t first, int64_t count,
                                  int8_t* accept_host, void* stream);

/* Copy the per-iteration log of the last solve of restart `restart`:
 * H_host[k] = H(x^(first+k)), r_host[k] = r^(first+k) for k < count.
 * Either output may be NULL.  Synchronous on `stream`.  Entries past the
 * restart's iters_done are undefined. */
ising_status ising_get_log(ising_ctx* ctx, int32_t restart, int64_t first,
                           int64_t count, double* H_host, double* r_host,
                           void* stream);

/* ----------------------------------------------------------------- energy
 * eq:IsingModel for R spin vectors:
 *   s_dev     int8[n * R] (interleaved, values +-1)
 *   E_dev     NULL or double[R]: -1/2 s^T J s - h^T s in FP64
 *   E_int_dev NULL or int64[R]: exact -1/2 s^T J s in integer arithmetic;
 *             requires integer couplings (ISING_E_UNSUPPORTED otherwise);
 *             the field term is not included.
 * Asynchronous on `stream`. */
ising_status ising_energy(ising_ctx* ctx, const int8_t* s_dev, int32_t R,
                          double* E_dev, int64_t* E_int_dev, void* stream);

/* ising_energy for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as ising_energy, but the partial sums
 * and arrival tickets live in a static device array of 4 MiB (one copy per
 * GPU, held until the process ends) instead of context memory that
 * ising_energy allocates on first use.  The call allocates and frees
 * nothing; the context itself is created beforehand as usual.  Every call
 * on one GPU shares that GPU's array, so calls that overlap in time on one
 * GPU (on different streams, or from different threads) race: serialise
 * them.  Tickets are cleared by a small kernel on `stream` at each call.
 * Errors: those of ising_energy; ISING_E_UNSUPPORTED for a batch context;
 * ISING_E_INVALID_ARG when the launch needs more partial sums than the
 * array holds (523 776 doubles: a CSR context takes any R <= 8, and
 * R <= 170 at any n; a stored dense context R < 8 at any n, and for
 * R >= 8 ceil(n/64) * ceil(R/64) * 128 partial sums; a generated dense
 * context 1024 * ceil(R/8) * 8 at n >= 4096, i.e. R <= 504).
 * Asynchronous on `stream`. */
ising_status ising_energy_noalloc(ising_ctx* ctx, const int8_t* s_dev, int32_t R,
                                  double* E_dev, int64_t* E_int_dev, void* stream);

/* MAX-CUT value of each spin vector (Supp. Note 5), for the graph whose edge
 * weights are the negated stored couplings, w_ij = -J_ij:
 *     cut(s) = sum over i < j with s_i != s_j of w_ij
 *            = -S_J / 4 - E(s) / 2,     S_J = sum of all stored J_ij,
 * with E(s) of eq:IsingModel.  The paper builds J = -W/2 from the weighted
 * adjacency matrix W; any positive multiple of -W gives the same DOCH
 * iterates under ising_default_params (alpha and beta scale with J), so a
 * graph with integer weights can be stored as J = -W (ISING_I16 fits the
 * 9-bit workload) and its cut read here in the weights' units.
 *   s_dev        int8[n x R] spins (+-1), restart-interleaved as for ising_energy
 *   cut_dev      NULL or R doubles
 *   cut_int_dev  NULL or R int64, exact; needs integer couplings (CSR)
 * Errors: ISING_E_UNSUPPORTED for a context with a field (the cut is defined
 * for h = 0), a batch context, or cut_int_dev on non-integer or dense
 * couplings; ISING_E_INVALID_ARG for NULL s_dev, R out of 1..1024 or no
 * output.  Asynchronous on `stream` except for a statistics pass that
 * synchronises it. */
ising_status ising_cut(ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* cut_dev,
                       int64_t* cut_int_dev, void* stream);

/* ------------------------------------------------- dense low precision
 * DOCH on a dense context for R restarts at once with J x computed on the
 * matrix cores: J is held in BF16 (jx_dtype = ISING_BF16) or in FP8 e4m3 with
 * one FP32 scale per row (ISING_FP8_E4M3), the restarts in FP32 plus a copy
 * in the same low precision, products accumulate in FP32.  The iteration
 * runs on u = sqrt(beta) x, where eq:FPE reads u <- cbrt(J u + alpha u)
 * exactly, so u stays representable in either format; the update forms
 * z + alpha u in FP64 and takes its cube root in FP32 (the precision u is
 * stored in).  H and r of each iteration (ising_get_log) are FP64 sums of the
 * low-precision products.  This solves a quantised problem: compare its
 * energies, not its iterates, with the FP64 path.
 *   x0_dev       double[n * R] (restart-interleaved, as ising_solve)
 *   params       alpha, beta, eps (per-restart freezing at r < eps); the
 *                iterate's storage fields are ignored
 *   x_out_dev    NULL or double[n * R]: final iterates x = u / sqrt(beta)
 *   s_out_dev    NULL or int8[n * R]: their signs (sign(0) = +1)
 *   H_final_dev  NULL or double[R]: H of the final iterates evaluated in FP64
 *                with the FP64 J (eq:Hamilton)
 *   stats_host   NULL or ising_stats[R]; makes the call synchronous.
 * Dense contexts without a field, n <= 65536, 1 <= R <= 1024. */
ising_status ising_solve_lowp(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t iters,
                              const ising_params* params, int32_t jx_dtype, double* x_out_dev,
                              int8_t* s_out_dev, double* H_final_dev, ising_stats* stats_host,
                              void* stream);

/* Shape of the matrix-core product of ising_solve_lowp on this context: each
 * iteration computes J U as tiles of 128 rows x bn restarts (bn = 64 or 128)
 * over `splits` equal parts of the k range (1, 2, 4 or 8), whose FP32
 * partial tiles the update adds in split order; the k range streams through
 * LDS in stages of stage_bytes per row (128 or 256) with `depth` stages in
 * flight (2 or 3).  splits = 0 selects the fused iteration instead: one
 * launch per iteration whose 64 x 64 tiles (bn 64, 256-byte stages) cover
 * the whole k range and update in place, with no partial tiles in memory;
 * splits = -1 runs that iteration resident, every iteration in one
 * cooperative launch with grid barriers between them (depth 2; when its
 * grid does not fit on the device at once, or for more than 10^8
 * iterations, the call runs the fused launches instead).  splits = -2
 * holds J in LDS for the whole run (bn 128, depth 1): one cooperative
 * launch of a workgroup per (128-row block, k slice of stage_bytes = 256,
 * 512 or 1024 bytes per row, at most 8 slices); per iteration every
 * workgroup multiplies its slice with the restart copy into FP32 partial
 * products, a grid barrier, the update adds the slices in order, a grid
 * barrier (when the workgroups do not fit on the device at once, or the run
 * is too long for the barrier's 32-bit counts -- 2 x iters x workgroups / 8
 * must stay below 2^31 -- the call runs the fused launches instead).  All
 * shapes compute the same products, in a different order of FP32
 * additions; the resident run and the fused launches are identical bit for
 * bit.  bn = 0 restores the default, the fused iteration (depth 3 in BF16
 * where the padded order holds three stages, else 2).  A shape that does
 * not fit a later call (bn not dividing the padded restart count, a split
 * holding fewer than `depth` whole stages, a held slice not dividing the
 * padded row or more than 8 slices) falls back to the default for that
 * call.  The shape changes the order of the FP32 additions, nothing else.
 * Errors: ISING_E_INVALID_ARG for a value outside those sets, for splits 0
 * or -1 with bn != 64 or stage_bytes != 256, or for splits -2 with bn !=
 * 128, depth != 1 or another slice width. */
ising_status ising_set_lowp_shape(ising_ctx* ctx, int32_t bn, int32_t splits, int32_t stage_bytes,
                                  int32_t depth);

/* Choose the shape of ising_solve_lowp for this context, restart count and
 * format by timing: every shape of ising_set_lowp_shape that fits (J held
 * in LDS over its slice widths, the fused iteration as launches and as a
 * resident run, and the split product over tile widths, splits, stage
 * widths and depths) runs `iters`
 * iterations from x0_dev twice, the second timed on `stream`; the fastest
 * becomes this context's shape.  With
 * cache_path non-NULL the choice is looked up first and stored after tuning
 * in a JSON file of one entry per line, keyed by device name, compute-unit
 * count, format, padded order, padded restart count and iters.
 *   shape_out       NULL or int32[4]: bn, splits (0 fused, -1 resident,
 *                   -2 J held in LDS), stage_bytes, depth
 *   ms_out          NULL or the chosen shape's time for `iters` iterations
 *   from_cache_out  NULL or 1 when the shape came from the cache
 * The context's last-solve state (logs, statistics) is overwritten.
 * Synchronises `stream`.  Errors: as ising_solve_lowp; ISING_E_INVALID_ARG
 * for iters < 1. */
ising_status ising_autotune_lowp(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t iters,
                                 const ising_params* params, int32_t jx_dtype, const char* cache_path, void* stream,
                                 int32_t* shape_out, double* ms_out, int32_t* from_cache_out);

/* ---------------------------------------------------------------- batches
 * Many independent instances solved together (the benchmark setting of the
 * paper's small and medium models: many instances and many random
 * initialisations).  The instances are the diagonal blocks of one CSR
 * matrix; instance k owns rows [r_k, r_k + n_k), r_k = n_0 + ... + n_{k-1},
 * and every coupling of those rows must lie in the same block.  No field.
 *
 * ising_create_batch: count >= 1 instances with n_host[k] >= 2 rows each;
 * row_ptr_dev / col_dev / val_dev / vt as for ising_create_csr over all
 * sum(n) rows with global column indices.  ISING_E_INVALID_ARG also when a
 * coupling leaves its block.  Synchronous.
 *
 * ising_default_params_batch: eq:alphabeta per instance (same rules as
 * ising_default_params, applied to each instance); alpha_host, beta_host
 * (and lambda_host when non-NULL) receive `count` values.  Synchronous.
 *
 * ising_solve_batch: DOCH on every instance with R restarts each (R in
 * {1, 2, 4, 8, 16, 32}) in one persistent kernel launch, replayed from a
 * captured HIP graph while the arguments repeat.  x0_dev is double[sum(n)*R]
 * (restart-interleaved), alpha_host / beta_host give each instance's
 * parameters, eps > 0 stops a restart at r^(k) < eps (its iterate is then
 * frozen) and an instance when all its restarts stopped, max_iters caps the
 * iterations; x_dtype stores the iterate in ISING_F64 or ISING_F32.
 * x_out_dev (double[sum(n)*R]) and s_out_dev (int8[sum(n)*R]) are optional.
 * stats_host (count*R entries, index k*R + r) and tts_ms_host (count
 * entries: milliseconds from the launch until instance k finished, from the
 * device clock) make the call synchronous; a synchronous call also returns
 * ISING_E_HIP if a team of workgroups gave up waiting at its barrier (after
 * about a second) or a restart was never run.  No per-iteration log.
 * With R <= 8 the instances' restart groups of rj restarts (units) are
 * dealt to the GPU's XCDs and each XCD iterates its units in lockstep: the
 * units' rows are cut into chunks of chunk_rows rows spread over all the
 * XCD's workgroups of wg threads, which meet at a barrier once per
 * iteration; a unit drops out when all its restarts stopped.  The shape
 * (rj, wg, chunk_rows) is set by ising_set_batch_shape or
 * ising_autotune_batch; default rj = 8 (or R), wg = 256 (512 below 4
 * restarts per unit), chunk_rows = 512.  The iterates do not depend on the
 * shape; H and r are summed in a shape-dependent order.
 *
 * ising_energy_batch: eq:IsingModel of each instance and restart,
 * E_dev[k*R + r] in FP64 and E_int_dev[k*R + r] exactly (integer couplings
 * only).  Asynchronous. */
ising_status ising_create_batch(int32_t count, const int64_t* n_host, const int32_t* row_ptr_dev,
                                const int32_t* col_dev, const void* val_dev, int32_t vt,
                                void* stream, ising_ctx** out);
ising_status ising_default_params_batch(ising_ctx* ctx, double eta, int32_t method,
                                        void* stream, double* alpha_host, double* beta_host,
                                        double* lambda_host);
ising_status ising_solve_batch(ising_ctx* ctx, const double* x0_dev, int32_t R,
                               int64_t max_iters, const double* alpha_host,
                               const double* beta_host, double eps, int32_t x_dtype,
                               double* x_out_dev, int8_t* s_out_dev, ising_stats* stats_host,
                               double* tts_ms_host, void* stream);
ising_status ising_energy_batch(ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* E_dev,
                                int64_t* E_int_dev, void* stream);

/* Launch shape of ising_solve_batch for R <= 8 (see above).  Built pairs
 * (rj, wg): (8, 256), (8, 512), (4, 256), (4, 512), (2, 512), (2, 1024),
 * (1, 512), (1, 1024); chunk_rows >= 1.  rj larger than the solve's R
 * runs R restarts per unit.  All three 0 restores the default.
 * ISING_E_INVALID_ARG for other values or a non-batch context. */
ising_status ising_set_batch_shape(ising_ctx* ctx, int32_t rj, int32_t wg, int32_t chunk_rows);

/* Choose the launch shape of ising_solve_batch for these arguments by
 * timing the solve (one warm-up and one timed run, device events) for every
 * built (rj <= R, wg) pair and chunk_rows in {256, 512, 1024, 2048}; the
 * fastest becomes the context's shape.  With cache_path, a JSON
 * file of earlier choices is consulted first, keyed by the device (gfx
 * name, CU count), the batch (instances, rows, couplings, value type) and
 * the solve (R, iterate type, max_iters, eps); a fresh choice is added to
 * it.  shape_out (3 ints: rj, wg, chunk_rows), ms_out (the chosen
 * shape's time in ms) and from_cache_out (1 when read from the file) may be
 * NULL.  The trial solves overwrite the context's iterate buffers and
 * statistics.  Arguments as for ising_solve_batch; R <= 8
 * (ISING_E_UNSUPPORTED above).  Synchronous. */
ising_status ising_autotune_batch(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t max_iters,
                                  const double* alpha_host, const double* beta_host, double eps,
                                  int32_t x_dtype, const char* cache_path, void* stream,
                                  int32_t* shape_out, double* ms_out, int32_t* from_cache_out);

/* ----------------------------------------------------------------- tuning
 * The CSR step kernel has several row-block geometries (see
 * ising_set_geometry).  They give identical results -- every row is summed
 * in ascending column order whatever the geometry -- and differ in speed.
 *
 * ising_set_geometry: 0 = 256-row blocks, 1024-entry spans; 1 = 512-row
 * blocks, 2048-entry spans; 2 = 512-row blocks, 4096-entry spans; 3 and 4 =
 * one row per lane with the whole grid sweeping the rows together, rows of
 * up to one (3) or two (4) aligned 4-entry chunks loaded at once (longer rows
 * take a slower path; with a constant row length, see ising_info.row_len,
 * the row offsets are implicit and not read; with small-integer values they
 * stream the library's compact copies, see ising_info.step_val_bytes and
 * step_col_bytes); 5, 6, 7 = geometries 0, 1, 2 with blocks handed out in
 * order from a per-XCD counter; 8 = resident: the whole single-restart DOCH
 * solve runs in one cooperative launch, with a grid-wide barrier between
 * iterations instead of a launch per iteration (for problems whose
 * iteration is shorter than a launch; it needs every workgroup of the launch
 * resident at once and fails with ISING_E_HIP if the device cannot hold
 * them); -1 = choose from the size and the mean row length (resident up to
 * 65536 rows and 2^20 stored entries).  wg_per_cu (0..32) caps the
 * workgroups launched per compute unit, 0 = as many as fit (ignored by
 * geometry 8).  Dense contexts take -1 (resident for stored matrices of order
 * up to 2048, else a launch per iteration), 0 (a launch per iteration) or 8
 * (resident; order up to 2048, stored matrices only).  Batch contexts take
 * none.  Every geometry gives the same iterates bit for bit.
 *
 * ising_autotune: time `iters` DOCH iterations (params as for ising_solve,
 * from x0_dev with R = 1; best of two timings) for every geometry and
 * workgroups-per-CU setting in {1, 2, 3, 4, all} (the resident geometry once,
 * up to 2^22 rows), and keep the fastest pair for later solves.
 * *geometry_out and *wg_per_cu_out (nullable) receive it, ms_per_iter_out
 * (nullable, 9 entries, 0 = not tried) the best time of each geometry.
 * Synchronous.  Overwrites the log of the last solve.  CSR contexts only. */
ising_status ising_set_geometry(ising_ctx* ctx, int32_t geometry, int32_t wg_per_cu);
ising_status ising_autotune(ising_ctx* ctx, const double* x0_dev, int64_t iters,
                            const ising_params* params, void* stream,
                            int32_t* geometry_out, int32_t* wg_per_cu_out,
                            double* ms_per_iter_out);

/* ------------------------------------------------------------------ misc */
const char* ising_status_string(ising_status s);
const char* ising_last_error(void);
/* Library version as "major.minor.patch". */
const char* ising_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ISING_H */
