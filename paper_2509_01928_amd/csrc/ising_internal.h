// ising_internal.h -- shared host-side declarations of the gfx950 DOCH
// library: the context object, the per-restart solver state and the kernel
// launchers implemented in the kernels_*.hip translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ising.h"

namespace doch {

// Row blocks of the CSR step kernel: a 256-thread workgroup handles up to
// `rows` consecutive rows whose stored entries lie within `span` entries of
// the block's first entry rounded down to a multiple of 4 (so they can be
// streamed as aligned 16-byte chunks).  A row that does not fit gets a block
// of its own and is reduced by the whole workgroup.
constexpr int kBlockThreads = 256;
// Column and value arrays are padded by this many entries so that a 16-byte
// chunk that starts before the last entry never reads past the allocation.
constexpr int kCsrPad = 4;
// Number of FP64 partial sums each workgroup contributes per restart and
// iteration: sum x^4, sum x^2, sum x*z, sum (x_new - x)^2, sum h*x.
constexpr int kNumPartials = 5;

// Device-resident state of one restart (one per column of an iterate block).
struct RestartState {
    int64_t iters_done;
    int32_t done;        // converged or failed: later iterations are skipped
    int32_t converged;
    int32_t nonfinite;
    int32_t aborted;     // a bounded wait of the resident solve ran out
    double H_last;
    double r_last;
};

// Reduced statistics of the coupling matrix (setup, eq:alphabeta).
struct MatrixStats {
    double rowsum_max;   // max_i sum_{j != i} |Jhat_ij|
    double abs_max;      // max_i sum_j |Jhat_ij| (power-method shift)
    double s1;           // sum_{i != j} Jhat_ij
    double ss;           // sum_{i != j} (Jhat_ij - mean)^2 over stored entries
    double stored;       // number of stored off-diagonal entries
    double pad[3];
};

struct CsrView {
    int64_t n;
    int64_t nnz;
    const int32_t* rp;
    const int32_t* col;
    const void* val;
    int vt;                 // ISING_F32 or ISING_F64
    const void* h;          // nullptr: no field
    int ht;
    int row_len;            // d > 0: every row holds d entries, row i starts at d i
    const int8_t* val8 = nullptr;  // the values as 8-bit integers when every one is an
                            // integer in [-128, 127] (padded like val), else nullptr
    const int16_t* col16 = nullptr;  // each entry's cyclic column offset col - i,
                            // taken into [-32768, 32767] modulo n, when every row
                            // holds 4 entries, val8 is kept and every offset fits
                            // (padded like col), else nullptr
};

struct DenseView {
    int64_t n;
    int64_t ld;
    const double* J;
    const void* h;
    int ht;
    int proc_kind;          // 0 = stored J, 1 = J_ij = sin(i j + seed)
    double proc_seed;
};

// A launch plan of the CSR step kernel.  Geometries 0-2 are row-block
// kernels (0: 256 rows and 1024-entry spans, 1: 512 rows / 2048, 2: 512 rows
// / 4096) whose blocks are stored as (first row, first entry) pairs;
// geometries 3 and 4 are lane-per-row kernels holding two rows per lane with
// rows of up to one (3) or two (4) aligned 16-byte chunks in registers;
// geometries 5-7 are 0-2 with blocks handed out in order by a per-XCD
// counter instead of a fixed stride.
// wg_per_cu caps the workgroups launched per CU (fewer resident workgroups
// interleave reads and writes less and can stream faster).
constexpr int kNumGeometries = 8;
// Block counters of the dynamically scheduled kernels sit this many uints
// apart (one 128-byte line each).
constexpr int kSchedStride = 32;
// Upper bound of a step kernel's grid (partial-sum buffers are sized for it).
constexpr int kMaxStepGrid = 8192;
struct CsrPlan {
    int geometry = 1;
    int2* binfo = nullptr;     // nblk + 1 entries
    int64_t nblk = 0;
    int wg_per_cu = 0;         // resident workgroups per CU to launch (0 = all that fit)
};

// Parameters of one DOCH iteration launch.
struct StepArgs {
    const void* x_old;      // n' * R, type x_dtype
    void* x_new;
    int x_dtype;            // ISING_F64 / ISING_F32
    int R;
    double alpha, beta, eps;
    int64_t k;              // iteration index
    double* partials;       // [grid][R][kNumPartials]
    unsigned int* ticket;
    unsigned int* sched;    // per-XCD block counters (kSchedStride apart), or nullptr
    double* log;            // [iters][R][2]: (H, r)
    RestartState* state;    // [R]
    int all_done_flag;      // unused placeholder
};

// ---- single-launch (resident) solves of small problems (kernels_resident.hip) ----
// Geometry id that selects the resident solve (CSR and dense contexts).
constexpr int kGeometryResident = 8;
// Largest dense order the resident solve holds in registers.
constexpr int64_t kResidentMaxDense = 2048;
// Row workgroups of a sparse resident solve (rows beyond 256 per workgroup
// take further passes).
constexpr int kResidentMaxCsrGroups = 255;
// Below these sizes a solve with the default geometry is resident.
constexpr int64_t kResidentAutoRows = 65536;
constexpr int64_t kResidentAutoNnz = 1 << 20;

// Barrier words of a resident solve; counters are 32 uints (one 128-byte
// line) apart.  grp[32 g]: arrivals of XCD group g; top[0]: groups complete;
// flag[32 g]: last barrier released to group g, flag[32 g + 1]: nonzero once
// the run stops (1 = finished early, 2 = a wait timed out).
struct ResidentSync {
    unsigned int grp[8 * 32];
    unsigned int top[32];
    unsigned int flag[8 * 32];
};

struct ResidentArgs {
    void* x;                // three iterate buffers, xstride elements apart;
    int64_t xstride;        // x^(k) is buffer k mod 3
    int x_dtype;
    int row_groups;         // workgroups owning rows; one more reduces
    double alpha, beta, eps;
    int64_t iters;
    double* partials;       // [2][row_groups][kNumPartials]
    double* log;            // [iters][2]: (H, r)
    RestartState* state;
    ResidentSync* sync;
};

// ADOCH (Alg. 2) on a stored dense matrix without a field, one restart, the
// whole run in one cooperative launch (kernels_resident.hip).
constexpr int kAdochResMaxW = 64;           // longest window q + 1 it keeps
constexpr int kAdochResPartials = 8;        // per workgroup: 7 sums, then 2
struct AdochResArgs {
    double* x;              // three FP64 iterate buffers, xstride apart; x^(k) in buffer k mod 3
    int64_t xstride;
    int row_groups;
    double alpha, beta, eps;
    int q;
    int64_t iters;
    const double* cseq;     // [iters] momentum weights c_k of Alg. 2
    double* partials;       // [3][row_groups][kAdochResPartials]
    double* log;            // [iters][2]: (H(x^(k)), r^(k))
    int8_t* accept_log;     // [iters]
    RestartState* state;
    ResidentSync* sync;
};

// ---- eta sweeps as restarts of one pass (kernels_sweep.hip) ----
constexpr int kSweepMaxR = 8;
struct SweepArgs {
    const double* x_old;    // (n' x R) restart-interleaved FP64 iterates
    double* x_new;
    int R;                  // 1..kSweepMaxR
    int64_t k;
    double alpha[kSweepMaxR], beta[kSweepMaxR];
    double* partials;       // [grid][R][kNumPartials]
    unsigned int* tickets;  // a grouped grid ticket (zero between launches)
    RestartState* state;    // [R]
};

// ---- batches of independent instances (kernels_batch.hip) ----
constexpr int kBatchThreads = 512;

// Instance k of a batch: rows [row0, row0 + n) of the block-diagonal CSR.
struct BatchInstance {
    int32_t row0;
    int32_t n;
    int32_t e0;
    int32_t nnz;
};

// Result of one restart of one instance.
struct BatchRestartStat {
    int64_t iters_done;
    int32_t converged;
    int32_t nonfinite;
    double H_last;
    double r_last;
};

// Launch shape of the dense low-precision product (launch_lowp_step).
struct LowpShape {
    int bn = 0, splits = 0, sb = 0, depth = 0;
};

// Launch shape of the batch solve for up to 8 restarts: restarts per unit
// of work (rj), threads per workgroup (wg) and rows per chunk (chunk_rows).
struct BatchShape {
    int rj = 8;
    int wg = 256;
    int chunk_rows = 512;
};

// A unit is restart group [r0, r0 + rj) of one instance; its rows are cut
// into nchunks chunks whose partial sums sit in slots first_slot.. of the
// plan's partial-sum array.
struct BatchUnit {
    int32_t inst, r0, first_slot, nchunks;
};
// Rows [lo, hi) of a unit; its partial sums go to slot `slot`.
struct BatchChunk {
    int32_t unit, lo, hi, slot;
};

constexpr int kBatchMaxXcd = 8;
// Counter words of the batch solve, each on its own 128-byte line:
// [32 x] workgroups registered on XCD x, [32 (8 + x)] its barrier,
// [32 (16 + x)] its finished units, [32 * 24] grid registration, [32 * 25] abort.
constexpr int kBatchCounterWords = 26 * 32;

// Device side of a batch plan (library-owned arrays built by the host).
struct BatchPlan {
    const BatchUnit* units = nullptr;
    const BatchChunk* chunks = nullptr;     // XCD x's chunks are [off[x], off[x + 1])
    const int32_t* off = nullptr;           // kBatchMaxXcd + 1 entries
    const int32_t* units_on = nullptr;      // kBatchMaxXcd entries: units per XCD
    int32_t n_units = 0;
    int32_t n_slots = 0;
    int32_t n_xcd = 1;
    int32_t rj = 1;
    unsigned int* counters = nullptr;       // kBatchCounterWords
    unsigned int* tickets = nullptr;        // per unit, 32 words apart
    int32_t* done = nullptr;                // per unit: iterations when it stopped, 0 while running
    int32_t* conv = nullptr;                // per unit and restart: stopped
    double* partials = nullptr;             // [slot][4 * rj]
};

// Arguments of the batch kernel for up to 8 restarts other than the row
// loop's pointers.  They live in device memory and the kernel reads them
// through one pointer (as kernel arguments they would hold scalar
// registers for the whole launch).
struct BatchStepArgs {
    const BatchInstance* inst;
    int R;
    const double* alpha;
    const double* beta;
    double eps;
    int64_t max_iters;
    const double* x0;
    BatchPlan plan;
    BatchRestartStat* stats;
    uint64_t* clock_start;
    uint64_t* clock_end;
    double* x_out;
    int8_t* s_out;
};

struct BatchView {
    int count;
    const int32_t* rp;
    const int32_t* col;
    const void* val;
    int vt;
    const BatchInstance* inst;
    const int32_t* order;     // instances by decreasing size
};

// Arguments of the two ADOCH launches of iteration k.
// Iterates of R restarts are interleaved: entry (i, r) at i R + r.
struct AdochArgs {
    double alpha, beta, eps;
    double c;                 // (t_k - 1) / t_{k+1}
    int64_t k;
    int q;                    // look-back window
    int R;                    // restarts: 1, 2, 4 or 8
    double* partials;
    unsigned int* ticket;
    double* log;              // [iters][R][2]: (H(x^(k)), r^(k))
    int* accept;              // [R]: decision of iteration k
    int* all_done;            // every restart stopped: later launches return at once
    int* fix;                 // [R] + word 8: fix-ups left by the optimistic CSR product
    int8_t* accept_log;       // [iters][R]
    double* ring;             // [R][q + 1]: last q+1 values of H(x)
    RestartState* state;      // [R]
};
constexpr int kAdochMaxR = 8;

}  // namespace doch

struct ising_ctx {
    int device = 0;
    bool dense = false;
    int64_t n = 0;
    int64_t np = 0;          // n' = n + has_field
    bool has_field = false;
    bool integer_J = false;
    // CSR storage (library-owned)
    int64_t nnz = 0;
    int32_t* rp = nullptr;
    int32_t* col = nullptr;
    void* val = nullptr;
    int8_t* val8 = nullptr;  // 8-bit copy of val read by the lane-per-row step
    int16_t* col16 = nullptr;  // 16-bit cyclic column offsets read by that step
    int vt = ISING_F32;
    void* h = nullptr;
    int ht = ISING_F32;
    // dense storage (or a procedural rule, proc_kind != 0)
    double* J = nullptr;
    int64_t ld = 0;
    int proc_kind = 0;
    double proc_seed = 0.0;
    // launch plans of the CSR step kernel, one per block geometry (built on
    // first use), and the geometry solves use (-1: chosen from the row lengths)
    doch::CsrPlan plans[doch::kNumGeometries];
    int geometry = -1;
    int wg_per_cu = 0;
    std::vector<int32_t> rp_host;
    // solve workspace
    void* xbuf[2] = {nullptr, nullptr};
    size_t xbuf_bytes = 0;
    double* partials = nullptr;
    size_t partials_bytes = 0;
    unsigned int* ticket = nullptr;
    doch::RestartState* state = nullptr;
    int state_cap = 0;
    double* log = nullptr;
    size_t log_bytes = 0;
    int last_R = 0;
    int64_t last_iters = 0;
    // setup scratch
    double* scratch = nullptr;
    size_t scratch_bytes = 0;
    // batch of instances (ising_create_batch)
    bool batch = false;
    int count = 0;
    doch::BatchInstance* inst = nullptr;
    int32_t* order = nullptr;
    std::vector<doch::BatchInstance> inst_host;
    double* bparams = nullptr;           // alpha[count], beta[count]
    doch::BatchRestartStat* bstats = nullptr;
    size_t bstats_bytes = 0;
    uint64_t* bclock = nullptr;          // [0] = start, [1 + k] = end of instance k
    unsigned int* bqueue = nullptr;
    // launch shape and job plan of the batch solve (R <= 8)
    doch::BatchShape bshape;
    bool bshape_set = false;
    std::vector<int64_t> bplan_key;
    doch::BatchPlan bplan;
    doch::BatchStepArgs bargs_host{};
    doch::BatchStepArgs* bargs_dev = nullptr;   // in bplan_mem
    void* bplan_mem = nullptr;
    size_t bplan_bytes = 0;
    // dense low-precision path (ising_solve_lowp)
    void* jq[2] = {nullptr, nullptr};    // BF16 / FP8 copies of J, padded
    float* rscale = nullptr;             // FP8 per-row scales
    double* rowabs = nullptr;            // FP8: s_i sum_j |q_ij| per row
    double lp_rho_q = 0.0;               // FP8: max_i rowabs[i]
    double* cut_tmp = nullptr;           // ising_cut: R energies, then R int64 energies
    int32_t row_len = 0;                 // CSR: constant row length d (rp[i] = d i), else 0
    double last_lambda = 0.0;            // lambda_hat and max row sum of the last
    double last_rowsum = 0.0;            // ising_default_params call
    int8_t* tune_s = nullptr;            // ising_tune_eta: rounded probe spins
    size_t tune_s_bytes = 0;
    double* sweep_x = nullptr;           // ising_tune_eta: two interleaved iterate blocks
    size_t sweep_x_bytes = 0;
    float* lp_cs = nullptr;              // FP8: restart scales, three buffers of kMaxR
    unsigned int* lp_colmax = nullptr;   // FP8: start column maxima (float bits)
    float* lp_u[3] = {nullptr, nullptr, nullptr};   // FP32 master iterates (rotating)
    void* lp_ub[3] = {nullptr, nullptr, nullptr};   // their low-precision copies
    size_t lp_ubytes = 0, lp_ubbytes = 0;
    double* lp_partials = nullptr;
    size_t lp_pbytes = 0;
    float* lp_P = nullptr;               // split partial products of one iteration
    size_t lp_Pbytes = 0;
    doch::LowpShape lp_shape;            // product shape set by the caller (bn 0: default)
    // ADOCH buffers (three iterates, two products, window, decisions)
    double* ad_x[3] = {nullptr, nullptr, nullptr};
    double* ad_z[2] = {nullptr, nullptr};
    size_t ad_bytes = 0;
    double* ad_ring = nullptr;
    int ad_ring_cap = 0;
    int* ad_accept = nullptr;
    int8_t* ad_acclog = nullptr;
    size_t ad_acclog_bytes = 0;
    double* ad_cseq = nullptr;           // momentum weights of a resident run
    size_t ad_cseq_bytes = 0;
    bool last_adoch = false;
    // resident solve: three iterate buffers and the barrier words
    void* rx = nullptr;
    size_t rx_bytes = 0;
    doch::ResidentSync* rsync = nullptr;
    // cached graph of the batch solve
    hipGraphExec_t bgraph = nullptr;
    hipGraph_t bgraph_src = nullptr;
    std::vector<uint64_t> bgraph_key;
};

namespace doch {

// ---- launchers (kernels_csr.hip) ----
hipError_t launch_csr_validate(const CsrView& A, int32_t* flags, hipStream_t s);
// out[0, nnz) = the values as 8-bit integers (valid when csr_validate
// raised no flags[3]); out must hold nnz + kCsrPad bytes
hipError_t launch_csr_pack_i8(const CsrView& A, int8_t* out, hipStream_t s);
// out[0, nnz) = every entry's cyclic column offset (valid when csr_validate
// raised no flags[4]); out must hold nnz + kCsrPad entries
hipError_t launch_csr_pack_col16(const CsrView& A, int16_t* out, hipStream_t s);
void csr_geometry(int geometry, int* rows, int* span);
hipError_t launch_csr_step(const CsrView& A, const CsrPlan& plan, const StepArgs& a,
                           hipStream_t s);
// workgroups of the one-pass energy for 2..8 restarts (its partials: 3 per
// workgroup and restart)
int csr_energy8_grid(int64_t n);
hipError_t launch_csr_energy(const CsrView& A, const int8_t* s_spins, int R,
                             double* partials, unsigned int* ticket, int grid,
                             double* E, int64_t* E_int, hipStream_t s);
hipError_t launch_csr_stats(const CsrView& A, double mean, int pass,
                            double* partials, unsigned int* ticket, int grid,
                            MatrixStats* out, hipStream_t s);
hipError_t launch_csr_power_step(const CsrView& A, double c, const double* v,
                                 double* w, double* partials, unsigned int* ticket,
                                 int grid, double* mu_log, int64_t k, hipStream_t s);
hipError_t launch_csr_symcheck(const CsrView& A, int32_t* bad, hipStream_t s);

// ---- launchers (kernels_dense.hip) ----
hipError_t launch_dense_validate(const DenseView& A, int32_t* flags, hipStream_t s);
hipError_t launch_dense_step(const DenseView& A, const StepArgs& a, int grid,
                             hipStream_t s);
int dense_step_grid(int64_t n);
// restarts from which ising_energy on a dense context uses the tiled J S kernel
constexpr int kTiledEnergyMinR = 8;
hipError_t launch_dense_energy(const DenseView& A, const int8_t* s_spins, int R,
                               double* partials, unsigned int* ticket, int grid,
                               double* E, hipStream_t s);
hipError_t launch_dense_stats(const DenseView& A, double mean, int pass,
                              double* partials, unsigned int* ticket, int grid,
                              MatrixStats* out, hipStream_t s);
hipError_t launch_dense_power_step(const DenseView& A, double c, const double* v,
                                   double* w, double* partials, unsigned int* ticket,
                                   int grid, double* mu_log, int64_t k, hipStream_t s);
hipError_t launch_dense_symcheck(const DenseView& A, int32_t* bad, hipStream_t s);

// ---- launchers (kernels_batch.hip) ----
bool batch_restarts_supported(int R);
hipError_t launch_batch_validate(const BatchView& B, int64_t n, int32_t* bad, hipStream_t s);
// Up to 8 restarts: every XCD iterates the units of its share of the plan
// in lockstep on a persistent grid of `wg`-thread workgroups; 16 or 32: one
// workgroup per instance with a restart per lane (shape and plan unused).
bool batch_shape_supported(const BatchShape& sh, int R);
// Resident workgroups of the shape's kernel on the current device.
int batch_shape_grid(const BatchShape& sh, int x_dtype, int vt);
// args_dev: the device copy of the kernel's arguments (R <= 8), written by
// the caller in stream order before the launch.
hipError_t launch_batch_solve(const BatchView& B, int R, const BatchShape& shape, const BatchPlan& plan,
                              const BatchStepArgs* args_dev, int64_t max_iters, const double* alpha,
                              const double* beta, double eps, int x_dtype, const double* x0,
                              void* xa, void* xb, unsigned int* queue, BatchRestartStat* stats,
                              uint64_t* clock_start, uint64_t* clock_end, double* x_out,
                              int8_t* s_out, hipStream_t s);
hipError_t launch_batch_energy(const BatchView& B, const int8_t* s_spins, int R, double* E,
                               int64_t* E_int, hipStream_t s);
hipError_t launch_batch_stats(const BatchView& B, double* out, hipStream_t s);
hipError_t launch_batch_power(const BatchView& B, const int32_t* jobs, int njobs,
                              const double* cshift, double tol, int64_t maxit, double* v, double* w,
                              double* lam, hipStream_t s);

// ---- launchers (kernels_mfma.hip) ----
hipError_t launch_lowp_convert(int prec, const double* J, int n, int np, void* Jq, float* rscale,
                               double* rowabs, hipStream_t s);
hipError_t launch_lowp_load(int prec, const double* x0, int n, int R, int np, int Rp, double sqrt_beta,
                            unsigned int* colmax_bits, float* cs, float* U, void* Ub, hipStream_t s);
// Shape of the product of one iteration: tiles of 128 rows x bn restarts
// (64 or 128), `splits` equal parts of the k range (1, 2, 4 or 8), stages of
// sb bytes per row (128 or 256) with `depth` stages in flight (2 or 3).
// Valid when the tiles divide the padded problem and every split holds at
// least `depth` whole stages.  splits 0 / -1: the fused iteration (64 x 64
// tiles, a launch per iteration / resident); splits -2: J held in LDS (bn
// 128 rows per block, sb = 256, 512 or 1024 k bytes per row per slice,
// depth 1), resident.
bool lowp_shape_valid(int prec, int np, int Rp, const LowpShape& sh);
LowpShape lowp_default_shape(int prec, int np, int Rp, int cus);
size_t lowp_product_bytes(int prec, int np, int Rp, const LowpShape& sh);   // the partial products P
// One iteration of the restart block: the split product into P, whose
// extra workgroups close iteration k - 1 from partials_prev (k > 0), then the
// update.  A stopped restart is never written, so its last iterate stays
// in buffer iters_done mod 3 (three buffers rotate).
hipError_t launch_lowp_step(int prec, int np, int Rp, const LowpShape& sh, const void* Jq, const float* rscale,
                            const float* U_old, float* U_new, const void* Ub_old, void* Ub_new,
                            const float* cs_old, float* cs_new, double rho_q, double alpha, double beta,
                            double eps, int R, int64_t k, float* P, const double* partials_prev,
                            double* partials, double* log, RestartState* state, hipStream_t s);
// The whole run of the fused iteration in one cooperative launch (shape
// splits -1): tiles resident on their compute units, grid barriers between
// iterations, each iteration closed by the next one's tiles (the last by
// launch_lowp_close).  sync must be zeroed (launch_resident_reset).
// hipErrorCooperativeLaunchTooLarge when the tiles do not fit on the device
// at once.
hipError_t launch_lowp_resident(int prec, int np, int Rp, const LowpShape& sh, int64_t iters, const void* Jq,
                                const float* rscale, float* const* U, void* const* Ub, float* const* cs,
                                double rho_q, double alpha, double beta, double eps, int R, double* const* partials,
                                double* log, RestartState* state, ResidentSync* sync, hipStream_t s);
// The whole run with J held in LDS (shape splits -2) in one cooperative
// launch: per iteration the split product into P, the closing of the
// previous iteration, a grid barrier, the update, a grid barrier.  P holds
// lowp_product_bytes; sync must be zeroed (launch_resident_reset); barrier
// arrivals are counted in 32-bit words (2 per iteration per workgroup of an
// XCD's share), so the caller keeps iters well below 2^31 / (workgroups /
// 8).  hipErrorCooperativeLaunchTooLarge when the workgroups do not fit on
// the device at once.
hipError_t launch_lowp_held(int prec, int np, int Rp, const LowpShape& sh, int64_t iters, const void* Jq,
                            const float* rscale, float* const* U, void* const* Ub, float* const* cs, double rho_q,
                            double alpha, double beta, double eps, int R, float* P, double* const* partials,
                            double* log, RestartState* state, ResidentSync* sync, hipStream_t s);
// Close iteration kk (the last one, after the final step).
hipError_t launch_lowp_close(int np, int Rp, int R, int64_t kk, const double* partials, double alpha,
                             double beta, double eps, double* log, RestartState* state, hipStream_t s);
hipError_t launch_lowp_finish(const float* const* U, const RestartState* state, int n, int R, int Rp,
                              double sqrt_beta, double* x_out, int8_t* s_out, hipStream_t s);
hipError_t launch_dense_objective(const double* J, int n, int R, const double* X, double alpha,
                                  double beta, double* partials, unsigned int* tickets, double* H,
                                  hipStream_t s);

// ---- launchers (kernels_adoch.hip, kernels_dense.hip) ----
// Workgroups of the ADOCH launches (partial sums: 7 R doubles per workgroup,
// 8 R for the optimistic CSR product).
int adoch_grid(int64_t n);
int adoch_dense_grid(const DenseView& A);
// xn non-null: the optimistic product, which writes x^(k+1) = T(y^(k)) and
// closes accepted restarts; follow it with launch_adoch_update(fixup = true).
hipError_t launch_adoch_mv(const CsrView& A, const double* x, const double* xp, const double* zp,
                           double* z, double* xn, const AdochArgs& a, hipStream_t s);
hipError_t launch_adoch_dense_mv(const DenseView& A, const double* x, const double* xp, const double* zp,
                                 double* z, const AdochArgs& a, hipStream_t s);
hipError_t launch_adoch_update(int64_t np, const double* x, const double* xp, const double* z,
                               const double* zp, double* xn, const AdochArgs& a, bool fixup, hipStream_t s);
// The resident ADOCH run above; hipErrorCooperativeLaunchTooLarge when its
// workgroups do not fit on the device at once.  sync must be zeroed.
hipError_t launch_resident_adoch_dense(const DenseView& A, const AdochResArgs& a, hipStream_t s);
hipError_t launch_adoch_finish(const double* b0, const double* b1, const double* b2,
                               const RestartState* st, int64_t n, int64_t np, int R, bool field,
                               double* x_out, int8_t* s_out, hipStream_t s);

// ---- launchers (kernels_resident.hip) ----
int resident_row_groups(bool dense, int64_t n);
hipError_t launch_resident_reset(ResidentSync* sy, hipStream_t s);
hipError_t launch_resident_dense(const DenseView& A, const ResidentArgs& a, hipStream_t s);
hipError_t launch_resident_csr(const CsrView& A, const ResidentArgs& a, hipStream_t s);

// ---- launchers (kernels_sweep.hip) ----
int sweep_grid(int64_t n);
hipError_t launch_sweep_step(const CsrView& A, const SweepArgs& a, hipStream_t s);
hipError_t launch_sweep_load(const double* x0, int64_t np, int R, double* X, hipStream_t s);
hipError_t launch_sweep_round(const double* X, int64_t n, int R, bool field, int8_t* S, hipStream_t s);
// the sweep on procedural couplings sin(i j + seed), 2 <= R <= 8, no field
int dense_sweep_grid(int64_t n);
hipError_t launch_dense_sin_sweep(int64_t n, double seed, const SweepArgs& a, hipStream_t s);

// ---- launchers (kernels_common.hip) ----
hipError_t launch_cut(const double* E, const int64_t* E_int, const MatrixStats* ms, int R, double* cut,
                      int64_t* cut_int, hipStream_t s);
hipError_t launch_load_x0(const double* x0, void* x, int x_dtype, int64_t count,
                          hipStream_t s);
hipError_t launch_init_state(RestartState* st, int R, unsigned int* ticket,
                             unsigned int* sched, hipStream_t s);
// xb2 == nullptr: the iterate alternates between xb0 and xb1; otherwise it
// rotates through all three.
hipError_t launch_finish(const void* xb0, const void* xb1, const void* xb2, int x_dtype,
                         const RestartState* st, int64_t n, int64_t np, int R,
                         bool field, double* x_out, int8_t* s_out, hipStream_t s);
hipError_t launch_normalize(const double* w, double* v, const double* mu_log,
                            int64_t k, int64_t n, hipStream_t s);

}  // namespace doch
