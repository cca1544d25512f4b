// api.hip -- the C ABI of include/ising.h: argument checking, ownership of
// device memory, the host-side DOCH loop (one kernel launch per iteration on
// the caller's stream) and the parameter setting of eq:alphabeta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ising_internal.h"

using doch::CsrView;
using doch::DenseView;
using doch::MatrixStats;
using doch::RestartState;
using doch::StepArgs;
using doch::BatchInstance;
using doch::BatchRestartStat;
using doch::BatchView;

namespace {

thread_local std::string g_last_error;

ising_status fail(ising_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

ising_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? ISING_E_OUT_OF_MEMORY : ISING_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_OK(call, what)                                       \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail(e_, what);         \
    } while (0)

size_t dtype_size(int t) {
    switch (t) {
        case ISING_F64: return 8;
        case ISING_F32: return 4;
        case ISING_BF16: return 2;
        case ISING_FP8_E4M3: return 1;
        case ISING_I32: return 4;
        case ISING_I16: return 2;
        default: return 0;
    }
}

bool float_dtype(int t) { return t == ISING_F32 || t == ISING_F64; }

template <typename T>
hipError_t dev_alloc(T** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    return hipMalloc(reinterpret_cast<void**>(p), bytes);
}

template <typename T>
void dev_free(T*& p) {
    if (p) (void)hipFree(static_cast<void*>(p));
    p = nullptr;
}

// Grow a workspace buffer to at least `bytes` (contents are not preserved).
template <typename T>
hipError_t ensure(T** p, size_t* cap, size_t bytes) {
    if (*p && *cap >= bytes) return hipSuccess;
    dev_free(*p);
    *cap = 0;
    hipError_t e = dev_alloc(p, bytes);
    if (e == hipSuccess) *cap = bytes;
    return e;
}

CsrView csr_view(const ising_ctx* c) {
    CsrView v;
    v.n = c->n;
    v.nnz = c->nnz;
    v.rp = c->rp;
    v.col = c->col;
    v.val = c->val;
    v.vt = c->vt;
    v.h = c->h;
    v.ht = c->ht;
    v.row_len = c->row_len;
    v.val8 = c->val8;
    v.col16 = c->col16;
    return v;
}

DenseView dense_view(const ising_ctx* c) {
    DenseView v;
    v.n = c->n;
    v.ld = c->ld;
    v.J = c->J;
    v.h = c->h;
    v.ht = c->ht;
    v.proc_kind = c->proc_kind;
    v.proc_seed = c->proc_seed;
    return v;
}

// Row blocks of the CSR step kernel for one geometry: consecutive rows, at
// most `rows` of them, whose entries end within `span` entries of the first
// entry rounded down to a multiple of 4; a row that does not fit alone is a
// block of its own.  Block b is stored as (first row, first entry) at b, with
// a sentinel (n, nnz) at the end.
std::vector<int2> make_blocks(const std::vector<int32_t>& rp, int64_t n, int rows, int span) {
    std::vector<int2> blk;
    blk.reserve(static_cast<size_t>(n / (rows / 2 + 1) + 2));
    int64_t r = 0;
    while (r < n) {
        const int64_t r0 = r;
        const int64_t ea = rp[r] & ~3;
        blk.push_back(make_int2(static_cast<int>(r0), rp[r0]));
        if (rp[r + 1] - ea > span) {
            r = r0 + 1;
        } else {
            while (r < n && r - r0 < rows && rp[r + 1] - ea <= span) ++r;
        }
    }
    blk.push_back(make_int2(static_cast<int>(n), rp[n]));
    return blk;
}

// Geometry from the mean row length: in-order scheduled row blocks of 512
// rows, 2048-entry spans for short rows and 4096-entry spans for long ones
// (the fastest on the lattice and random-graph workloads measured).
// Short rows (lattices, mean length up to 5): one row per lane; longer rows:
// row blocks from per-XCD counters.
// Small problems (up to 65536 rows and 2^20 entries) run resident: the whole
// solve in one cooperative launch, since a launch per iteration would cost
// more than the iteration.
int default_geometry(int64_t n, int64_t nnz) {
    if (n <= doch::kResidentAutoRows && nnz <= doch::kResidentAutoNnz) return doch::kGeometryResident;
    const double d = static_cast<double>(nnz) / static_cast<double>(n);
    return d <= 5.0 ? 4 : (d <= 8.0 ? 6 : 7);
}

// Kernels that read row offsets hide their dependent load chains with as
// many resident workgroups as fit; with 4-entry rows and implicit offsets
// (no chain) four per CU stream fastest with 32-bit column indices
// (measured on gfx950, 10^8-spin lattice: 795 us against 878 us with all
// that fit; 624 against 628 with 8-bit values), but with the 16-bit column
// offsets all that fit are fastest again (546 us against 554 with six, 580
// with five, 628 with four).
int default_wg_per_cu(int geometry, int row_len, bool col16) {
    return ((geometry == 3 || geometry == 4) && row_len == 4 && !col16) ? 4 : 0;
}

ising_status ensure_plan(ising_ctx* c, int geometry, doch::CsrPlan** out) {
    doch::CsrPlan& p = c->plans[geometry];
    int rows = 0, span = 0;
    doch::csr_geometry(geometry, &rows, &span);
    if (rows == 0) {                 // lane-per-row kernels need no block table
        p.geometry = geometry;
        p.nblk = c->n;
    } else if (!p.binfo) {
        std::vector<int2> blk = make_blocks(c->rp_host, c->n, rows, span);
        p.geometry = geometry;
        p.nblk = static_cast<int64_t>(blk.size()) - 1;
        HIP_OK(dev_alloc(&p.binfo, blk.size() * sizeof(int2)), "hipMalloc(blocks)");
        HIP_OK(hipMemcpy(p.binfo, blk.data(), blk.size() * sizeof(int2), hipMemcpyHostToDevice),
               "copy blocks");
    }
    *out = &p;
    return ISING_OK;
}

void free_ctx(ising_ctx* c) {
    if (!c) return;
    dev_free(c->rp);
    dev_free(c->col);
    dev_free(c->val);
    dev_free(c->val8);
    dev_free(c->col16);
    dev_free(c->h);
    dev_free(c->J);
    for (auto& p : c->plans) dev_free(p.binfo);
    dev_free(c->xbuf[0]);
    dev_free(c->xbuf[1]);
    dev_free(c->partials);
    dev_free(c->ticket);
    dev_free(c->state);
    dev_free(c->log);
    dev_free(c->scratch);
    dev_free(c->inst);
    dev_free(c->order);
    dev_free(c->bparams);
    dev_free(c->bstats);
    dev_free(c->bclock);
    dev_free(c->bqueue);
    dev_free(c->bplan_mem);
    dev_free(c->jq[0]);
    dev_free(c->jq[1]);
    dev_free(c->rscale);
    dev_free(c->rowabs);
    dev_free(c->cut_tmp);
    dev_free(c->tune_s);
    dev_free(c->sweep_x);
    dev_free(c->lp_cs);
    dev_free(c->lp_colmax);
    for (auto& b : c->lp_u) dev_free(b);
    for (auto& b : c->lp_ub) dev_free(b);
    dev_free(c->lp_partials);
    dev_free(c->lp_P);
    dev_free(c->rx);
    dev_free(c->rsync);
    for (auto& b : c->ad_x) dev_free(b);
    for (auto& b : c->ad_z) dev_free(b);
    dev_free(c->ad_ring);
    dev_free(c->ad_accept);
    dev_free(c->ad_acclog);
    dev_free(c->ad_cseq);
    if (c->bgraph) (void)hipGraphExecDestroy(c->bgraph);
    if (c->bgraph_src) (void)hipGraphDestroy(c->bgraph_src);
    delete c;
}

ising_status copy_field(ising_ctx* c, const void* h_dev, int32_t ht, hipStream_t s) {
    if (!h_dev) return ISING_OK;
    if (!float_dtype(ht)) return fail(ISING_E_INVALID_ARG, "field dtype must be ISING_F32 or ISING_F64");
    const size_t bytes = static_cast<size_t>(c->n) * dtype_size(ht);
    HIP_OK(dev_alloc(&c->h, bytes), "hipMalloc(h)");
    HIP_OK(hipMemcpyAsync(c->h, h_dev, bytes, hipMemcpyDeviceToDevice, s), "copy h");
    c->ht = ht;
    c->has_field = true;
    c->np = c->n + 1;
    return ISING_OK;
}

// Scratch of the context (setup, energy): flags, tickets and partial sums.
struct Scratch {
    int32_t* flags;           // 8 ints
    unsigned int* tickets;    // 1024
    MatrixStats* stats;       // 1
    double* mu_log;           // 2 * kPowerChunk
    double* vecs;             // 2 * np (power iteration)
    double* partials;         // rest
    size_t partial_doubles;
};

constexpr int kPowerChunk = 64;
// The autotuner tries the resident solve up to this many rows (beyond, each
// lane walks thousands of rows per iteration and the streaming kernels win).
constexpr int64_t kResidentTuneMaxRows = 1 << 22;
constexpr int kMaxR = 1024;

ising_status ensure_scratch(ising_ctx* c, size_t partial_doubles, Scratch* out) {
    const size_t head = 256 + kMaxR * sizeof(unsigned int) + sizeof(MatrixStats) +
                        2 * kPowerChunk * sizeof(double);
    const size_t vec_bytes = 2 * static_cast<size_t>(c->np) * sizeof(double);
    const size_t need = head + vec_bytes + partial_doubles * sizeof(double) + 256;
    if (!c->scratch || c->scratch_bytes < need) {
        dev_free(c->scratch);
        c->scratch_bytes = 0;
        HIP_OK(dev_alloc(&c->scratch, need), "hipMalloc(scratch)");
        HIP_OK(hipMemset(c->scratch, 0, need), "hipMemset(scratch)");
        c->scratch_bytes = need;
    }
    char* base = reinterpret_cast<char*>(c->scratch);
    out->flags = reinterpret_cast<int32_t*>(base);
    out->tickets = reinterpret_cast<unsigned int*>(base + 256);
    out->stats = reinterpret_cast<MatrixStats*>(base + 256 + kMaxR * sizeof(unsigned int));
    out->mu_log = reinterpret_cast<double*>(base + 256 + kMaxR * sizeof(unsigned int) +
                                            sizeof(MatrixStats));
    out->vecs = out->mu_log + 2 * kPowerChunk;
    out->partials = out->vecs + 2 * c->np;
    out->partial_doubles = partial_doubles;
    return ISING_OK;
}

}  // namespace

// Per-restart state, tickets and the (H, r) log of a solve of `iters`
// iterations and R restarts.
static ising_status ensure_solve_state(ising_ctx* ctx, int64_t iters, int R) {
    if (!ctx->ticket) {
        HIP_OK(dev_alloc(&ctx->ticket, (kMaxR + 8 * doch::kSchedStride) * sizeof(unsigned int)),
               "hipMalloc(ticket)");
        HIP_OK(dev_alloc(&ctx->state, kMaxR * sizeof(RestartState)), "hipMalloc(state)");
        ctx->state_cap = kMaxR;
    }
    HIP_OK(ensure(&ctx->log, &ctx->log_bytes, static_cast<size_t>(std::max<int64_t>(iters, 1)) * R * 2 * sizeof(double)),
           "hipMalloc(log)");
    return ISING_OK;
}

// Copy the restarts' state into stats_host (if given; synchronises).
static ising_status read_stats(ising_ctx* ctx, int R, ising_stats* stats_host, hipStream_t s) {
    if (!stats_host) return ISING_OK;
    std::vector<RestartState> hs(static_cast<size_t>(R));
    HIP_OK(hipMemcpyAsync(hs.data(), ctx->state, R * sizeof(RestartState), hipMemcpyDeviceToHost, s),
           "copy state");
    HIP_OK(hipStreamSynchronize(s), "sync");
    bool bad = false, aborted = false;
    for (int r = 0; r < R; ++r) {
        stats_host[r].iters_done = hs[r].iters_done;
        stats_host[r].converged = hs[r].converged;
        stats_host[r].nonfinite = hs[r].nonfinite;
        stats_host[r].H_last = hs[r].H_last;
        stats_host[r].r_last = hs[r].r_last;
        bad = bad || hs[r].nonfinite;
        aborted = aborted || hs[r].aborted;
    }
    if (aborted) return fail(ISING_E_HIP, "a grid barrier wait of the resident solve timed out");
    if (bad) return fail(ISING_E_NONFINITE, "H or r became non-finite");
    return ISING_OK;
}

// Whether a single-restart DOCH solve of this context runs resident (one
// cooperative launch for all iterations): a CSR context set to the resident
// geometry, or a stored dense matrix of order up to 2048 unless another
// geometry was set.
static bool resident_selected(const ising_ctx* ctx) {
    if (ctx->dense)
        return ctx->proc_kind == 0 && ctx->n <= doch::kResidentMaxDense &&
               (ctx->geometry == doch::kGeometryResident || ctx->geometry < 0);
    return ctx->geometry == doch::kGeometryResident;
}

// The whole solve in one cooperative launch (kernels_resident.hip).
static ising_status solve_resident(ising_ctx* ctx, const double* x0_dev, int64_t iters, const ising_params& p,
                                   double* x_out_dev, int8_t* s_out_dev, ising_stats* stats_host, hipStream_t s) {
    // three iterate buffers in one allocation, each rounded up to 256 bytes
    const int64_t elt = p.x_dtype == ISING_F64 ? 8 : 4;
    const int64_t xstride = (ctx->np * elt + 255) / 256 * 256 / elt;
    const size_t xbytes = 3 * static_cast<size_t>(xstride) * elt;
    HIP_OK(ensure(&ctx->rx, &ctx->rx_bytes, xbytes), "hipMalloc(x)");
    char* rx = static_cast<char*>(ctx->rx);
    void* xb[3] = {rx, rx + xstride * elt, rx + 2 * xstride * elt};
    const int G = doch::resident_row_groups(ctx->dense, ctx->n);
    HIP_OK(ensure(&ctx->partials, &ctx->partials_bytes, 2 * static_cast<size_t>(G) * doch::kNumPartials * sizeof(double)),
           "hipMalloc(partials)");
    ising_status sst = ensure_solve_state(ctx, iters, 1);
    if (sst != ISING_OK) return sst;
    if (!ctx->rsync) HIP_OK(dev_alloc(&ctx->rsync, sizeof(doch::ResidentSync)), "hipMalloc(sync)");
    HIP_OK(doch::launch_init_state(ctx->state, 1, ctx->ticket, ctx->ticket + kMaxR, s), "init");
    HIP_OK(doch::launch_resident_reset(ctx->rsync, s), "reset");
    HIP_OK(doch::launch_load_x0(x0_dev, xb[0], p.x_dtype, ctx->np, s), "load x0");
    doch::ResidentArgs a;
    a.x = ctx->rx;
    a.xstride = xstride;
    a.x_dtype = p.x_dtype;
    a.row_groups = G;
    a.alpha = p.alpha;
    a.beta = p.beta;
    a.eps = p.eps;
    a.iters = iters;
    a.partials = ctx->partials;
    a.log = ctx->log;
    a.state = ctx->state;
    a.sync = ctx->rsync;
    if (iters > 0) {
        const hipError_t e = ctx->dense ? doch::launch_resident_dense(dense_view(ctx), a, s)
                                        : doch::launch_resident_csr(csr_view(ctx), a, s);
        if (e != hipSuccess) return hip_fail(e, "resident solve launch");
    }
    ctx->last_R = 1;
    ctx->last_iters = iters;
    ctx->last_adoch = false;
    if (x_out_dev || s_out_dev)
        HIP_OK(doch::launch_finish(xb[0], xb[1], xb[2], p.x_dtype, ctx->state, ctx->n, ctx->np, 1,
                                   ctx->has_field, x_out_dev, s_out_dev, s), "finish");
    return read_stats(ctx, 1, stats_host, s);
}

// ADOCH (Alg. 2) on a single CSR or dense (stored or generated) context,
// R in {1, 2, 4, 8} interleaved restarts, FP64 iterates.
static ising_status solve_adoch(ising_ctx* ctx, const double* x0_dev, int R, int64_t iters, const ising_params& p,
                         double* x_out_dev, int8_t* s_out_dev, ising_stats* stats_host, hipStream_t s) {
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t bytes = static_cast<size_t>(ctx->np) * R * sizeof(double);
    if (!ctx->ad_x[0] || ctx->ad_bytes < bytes) {
        for (auto& b : ctx->ad_x) dev_free(b);
        for (auto& b : ctx->ad_z) dev_free(b);
        ctx->ad_bytes = 0;
        for (auto& b : ctx->ad_x) HIP_OK(dev_alloc(&b, bytes), "hipMalloc(x)");
        for (auto& b : ctx->ad_z) HIP_OK(dev_alloc(&b, bytes), "hipMalloc(z)");
        ctx->ad_bytes = bytes;
    }
    if (!ctx->ad_ring || ctx->ad_ring_cap < R * (p.q + 1)) {
        dev_free(ctx->ad_ring);
        HIP_OK(dev_alloc(&ctx->ad_ring, static_cast<size_t>(R) * (p.q + 1) * sizeof(double)), "hipMalloc(ring)");
        ctx->ad_ring_cap = R * (p.q + 1);
    }
    // decisions [R], the fix-up marks (words 16 to 24) and the all-done flag (word 64)
    if (!ctx->ad_accept) HIP_OK(dev_alloc(&ctx->ad_accept, 512), "hipMalloc(accept)");
    HIP_OK(ensure(&ctx->ad_acclog, &ctx->ad_acclog_bytes, static_cast<size_t>(std::max<int64_t>(iters, 1)) * R),
           "hipMalloc(accept log)");
    // momentum sequence of Alg. 2: t_0 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
    // c_k = (t_k - 1) / t_{k+1} (0 at k = 0: y^(0) = x^(0))
    auto momentum = [](int64_t k, double* t) {
        const double t_next = (1.0 + std::sqrt(1.0 + 4.0 * *t * *t)) / 2.0;
        const double c = (*t - 1.0) / t_next;
        *t = t_next;
        (void)k;
        return c;
    };
    const int mv_grid = ctx->dense ? doch::adoch_dense_grid(dense_view(ctx)) : doch::adoch_grid(ctx->n);
    const int up_grid = doch::adoch_grid(ctx->np * R);
    const size_t pd = std::max(static_cast<size_t>(mv_grid) * 8 * R, static_cast<size_t>(up_grid) * 2 * R);
    HIP_OK(ensure(&ctx->partials, &ctx->partials_bytes, pd * sizeof(double)), "hipMalloc(partials)");
    if (!ctx->ticket) {
        HIP_OK(dev_alloc(&ctx->ticket, (kMaxR + 8 * doch::kSchedStride) * sizeof(unsigned int)), "hipMalloc(ticket)");
        HIP_OK(dev_alloc(&ctx->state, kMaxR * sizeof(RestartState)), "hipMalloc(state)");
        ctx->state_cap = kMaxR;
    }
    HIP_OK(ensure(&ctx->log, &ctx->log_bytes,
                  static_cast<size_t>(std::max<int64_t>(iters, 1)) * R * 2 * sizeof(double)), "hipMalloc(log)");
    // a stored dense matrix of order <= 2048 without a field, one restart:
    // the whole run in one cooperative launch, unless another geometry was
    // set (barrier arrivals are counted in 32-bit words: at most 10^7
    // iterations)
    if (ctx->dense && ctx->proc_kind == 0 && !ctx->has_field && R == 1 && ctx->n <= doch::kResidentMaxDense &&
        p.q + 1 <= doch::kAdochResMaxW && iters > 0 && iters <= 10000000 &&
        (ctx->geometry == doch::kGeometryResident || ctx->geometry < 0)) {
        const int64_t xstride = (ctx->np * 8 + 255) / 256 * 256 / 8;
        HIP_OK(ensure(&ctx->rx, &ctx->rx_bytes, 3 * static_cast<size_t>(xstride) * 8), "hipMalloc(x)");
        double* rx = static_cast<double*>(ctx->rx);
        const int G = doch::resident_row_groups(true, ctx->n);
        HIP_OK(ensure(&ctx->partials, &ctx->partials_bytes,
                      3 * static_cast<size_t>(G) * doch::kAdochResPartials * sizeof(double)), "hipMalloc(partials)");
        // c_0 .. c_{iters-1}, kept on the device for later runs (the whole
        // allocation always holds the sequence from k = 0)
        const size_t cbytes = static_cast<size_t>(iters) * sizeof(double);
        if (!ctx->ad_cseq || ctx->ad_cseq_bytes < cbytes) {
            std::vector<double> cs(static_cast<size_t>(iters));
            double t = 1.0;
            for (int64_t k = 0; k < iters; ++k) cs[static_cast<size_t>(k)] = momentum(k, &t);
            HIP_OK(ensure(&ctx->ad_cseq, &ctx->ad_cseq_bytes, cbytes), "hipMalloc(c)");
            HIP_OK(hipMemcpyAsync(ctx->ad_cseq, cs.data(), cbytes, hipMemcpyHostToDevice, s), "copy c");
            HIP_OK(hipStreamSynchronize(s), "sync");        // cs is released here
        }
        if (!ctx->rsync) HIP_OK(dev_alloc(&ctx->rsync, sizeof(doch::ResidentSync)), "hipMalloc(sync)");
        HIP_OK(doch::launch_init_state(ctx->state, 1, ctx->ticket, nullptr, s), "init");
        HIP_OK(doch::launch_resident_reset(ctx->rsync, s), "reset");
        HIP_OK(hipMemcpyAsync(rx, x0_dev, bytes, hipMemcpyDeviceToDevice, s), "load x0");
        doch::AdochResArgs ra;
        ra.x = rx;
        ra.xstride = xstride;
        ra.row_groups = G;
        ra.alpha = p.alpha;
        ra.beta = p.beta;
        ra.eps = p.eps;
        ra.q = p.q;
        ra.iters = iters;
        ra.cseq = ctx->ad_cseq;
        ra.partials = ctx->partials;
        ra.log = ctx->log;
        ra.accept_log = ctx->ad_acclog;
        ra.state = ctx->state;
        ra.sync = ctx->rsync;
        const hipError_t e = doch::launch_resident_adoch_dense(dense_view(ctx), ra, s);
        if (e == hipSuccess) {
            ctx->last_R = 1;
            ctx->last_iters = iters;
            ctx->last_adoch = true;
            if (x_out_dev || s_out_dev)
                HIP_OK(doch::launch_adoch_finish(rx, rx + xstride, rx + 2 * xstride, ctx->state, ctx->n, ctx->np, 1,
                                                 false, x_out_dev, s_out_dev, s), "finish");
            return read_stats(ctx, 1, stats_host, s);
        }
        if (e != hipErrorCooperativeLaunchTooLarge) return hip_fail(e, "resident ADOCH launch");
        (void)hipGetLastError();
    }
    HIP_OK(doch::launch_init_state(ctx->state, R, ctx->ticket, nullptr, s), "init");
    HIP_OK(hipMemsetAsync(ctx->ad_accept, 0, 512, s), "clear flags");
    HIP_OK(hipMemcpyAsync(ctx->ad_x[0], x0_dev, bytes, hipMemcpyDeviceToDevice, s), "load x0");
    // z^(-1) enters with weight c_0 = 0; it must be finite
    HIP_OK(hipMemsetAsync(ctx->ad_z[1], 0, bytes, s), "clear z");
    doch::AdochArgs a;
    a.alpha = p.alpha;
    a.beta = p.beta;
    a.eps = p.eps;
    a.q = p.q;
    a.R = R;
    a.partials = ctx->partials;
    a.ticket = ctx->ticket;
    a.log = ctx->log;
    a.accept = ctx->ad_accept;
    a.all_done = ctx->ad_accept + 64;
    a.fix = ctx->ad_accept + 16;
    a.accept_log = ctx->ad_acclog;
    a.ring = ctx->ad_ring;
    a.state = ctx->state;
    const CsrView cv = csr_view(ctx);
    const DenseView dv = dense_view(ctx);
    double t = 1.0;
    for (int64_t k = 0; k < iters; ++k) {
        a.c = momentum(k, &t);
        a.k = k;
        const double* x = ctx->ad_x[k % 3];
        const double* xp = k == 0 ? ctx->ad_x[0] : ctx->ad_x[(k + 2) % 3];
        double* xn = ctx->ad_x[(k + 1) % 3];
        double* z = ctx->ad_z[k % 2];
        const double* zp = ctx->ad_z[(k + 1) % 2];
        // CSR: the product writes x^(k+1) of an accepted y itself; the update
        // launch only repairs rejected restarts (and returns at once if none)
        if (ctx->dense)
            HIP_OK(doch::launch_adoch_dense_mv(dv, x, xp, zp, z, a, s), "ADOCH matvec");
        else
            HIP_OK(doch::launch_adoch_mv(cv, x, xp, zp, z, xn, a, s), "ADOCH matvec");
        HIP_OK(doch::launch_adoch_update(ctx->np, x, xp, z, zp, xn, a, !ctx->dense, s), "ADOCH update");
    }
    ctx->last_R = R;
    ctx->last_iters = iters;
    ctx->last_adoch = true;
    if (x_out_dev || s_out_dev)
        HIP_OK(doch::launch_adoch_finish(ctx->ad_x[0], ctx->ad_x[1], ctx->ad_x[2], ctx->state, ctx->n, ctx->np, R,
                                         ctx->has_field, x_out_dev, s_out_dev, s), "finish");
    return read_stats(ctx, R, stats_host, s);
}

namespace {
bool cache_lookup_ints(const char* path, const std::string& key, const char* const* names, int n, int* vals,
                       double* ms);
bool cache_store_ints(const char* path, const std::string& key, const char* const* names, int n, const int* vals,
                      double ms);
extern const char* const kLowpFields[4];
}  // namespace

extern "C" {

const char* ising_version(void) { return "0.1.0"; }

ising_status ising_get_accept_log(ising_ctx* ctx, int64_t first, int64_t count, int8_t* accept_host,
                                  void* stream) {
    if (!ctx || !accept_host) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (!ctx->last_adoch) return fail(ISING_E_INVALID_ARG, "the last solve was not ADOCH");
    if (first < 0 || count < 0 || first + count > ctx->last_iters) return fail(ISING_E_INVALID_ARG, "bad range");
    if (count == 0) return ISING_OK;
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int R = ctx->last_R;
    HIP_OK(hipMemcpyAsync(accept_host, ctx->ad_acclog + first * R, static_cast<size_t>(count) * R,
                          hipMemcpyDeviceToHost, s), "copy");
    HIP_OK(hipStreamSynchronize(s), "sync");
    return ISING_OK;
}

const char* ising_last_error(void) { return g_last_error.c_str(); }

const char* ising_status_string(ising_status s) {
    switch (s) {
        case ISING_OK: return "ok";
        case ISING_E_INVALID_ARG: return "invalid argument";
        case ISING_E_NONZERO_DIAG: return "nonzero diagonal coupling";
        case ISING_E_NOT_SYMMETRIC: return "coupling matrix is not symmetric";
        case ISING_E_OUT_OF_MEMORY: return "out of device memory";
        case ISING_E_HIP: return "HIP runtime error";
        case ISING_E_UNSUPPORTED: return "unsupported request";
        case ISING_E_NONFINITE: return "non-finite objective";
    }
    return "unknown status";
}

ising_status ising_create_csr(int64_t n, int64_t nnz, const int32_t* row_ptr_dev,
                              const int32_t* col_dev, const void* val_dev, int32_t vt,
                              const void* h_dev, int32_t ht, void* stream, ising_ctx** out) {
    if (!out) return fail(ISING_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= 2147483647LL) return fail(ISING_E_INVALID_ARG, "n=%lld out of range", (long long)n);
    if (nnz < 0 || nnz >= 2147483647LL) return fail(ISING_E_INVALID_ARG, "nnz=%lld out of range", (long long)nnz);
    if (!row_ptr_dev) return fail(ISING_E_INVALID_ARG, "row_ptr is NULL");
    if (nnz > 0 && (!col_dev || !val_dev)) return fail(ISING_E_INVALID_ARG, "col/val NULL with nnz > 0");
    if (!float_dtype(vt) && vt != ISING_I16)
        return fail(ISING_E_INVALID_ARG, "CSR values must be ISING_F32, ISING_F64 or ISING_I16");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ising_ctx* c = new ising_ctx();
    ising_status st = ISING_OK;
    auto bail = [&](ising_status e) { free_ctx(c); return e; };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(ISING_E_HIP, "no HIP device"));
    c->dense = false;
    c->n = n;
    c->np = n;
    c->nnz = nnz;
    c->vt = vt;
    hipError_t e;
    if ((e = dev_alloc(&c->rp, (n + 1) * sizeof(int32_t))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(rp)"));
    const int64_t padded = nnz + doch::kCsrPad;
    if ((e = dev_alloc(&c->col, padded * sizeof(int32_t))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(col)"));
    if ((e = dev_alloc(&c->val, padded * dtype_size(vt))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(val)"));
    if ((e = hipMemsetAsync(c->col + nnz, 0, doch::kCsrPad * sizeof(int32_t), s)) != hipSuccess)
        return bail(hip_fail(e, "memset pad"));
    if ((e = hipMemsetAsync(static_cast<char*>(c->val) + nnz * dtype_size(vt), 0, doch::kCsrPad * dtype_size(vt), s)) !=
        hipSuccess)
        return bail(hip_fail(e, "memset pad"));
    if ((e = hipMemcpyAsync(c->rp, row_ptr_dev, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return bail(hip_fail(e, "copy row_ptr"));
    if (nnz > 0) {
        if ((e = hipMemcpyAsync(c->col, col_dev, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return bail(hip_fail(e, "copy col"));
        if ((e = hipMemcpyAsync(c->val, val_dev, nnz * dtype_size(vt), hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return bail(hip_fail(e, "copy val"));
    }
    if ((st = copy_field(c, h_dev, ht, s)) != ISING_OK) return bail(st);
    Scratch sc;
    if ((st = ensure_scratch(c, 0, &sc)) != ISING_OK) return bail(st);
    if ((e = hipMemsetAsync(sc.flags, 0, 8 * sizeof(int32_t), s)) != hipSuccess) return bail(hip_fail(e, "memset"));
    if ((e = doch::launch_csr_validate(csr_view(c), sc.flags, s)) != hipSuccess) return bail(hip_fail(e, "validate"));
    int32_t flags[8];
    if ((e = hipMemcpyAsync(flags, sc.flags, sizeof(flags), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return bail(hip_fail(e, "copy flags"));
    std::vector<int32_t> rp_host(static_cast<size_t>(n + 1));
    if ((e = hipMemcpyAsync(rp_host.data(), c->rp, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return bail(hip_fail(e, "copy row_ptr to host"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "sync"));
    if (rp_host[0] != 0 || rp_host[n] != nnz) flags[0] = 1;
    for (int64_t i = 0; i < n && !flags[0]; ++i)
        if (rp_host[i + 1] < rp_host[i]) flags[0] = 1;
    if (flags[0]) return bail(fail(ISING_E_INVALID_ARG, "malformed CSR (offsets, column range or order)"));
    if (flags[1]) return bail(fail(ISING_E_NONZERO_DIAG, "a diagonal coupling J_ii is nonzero"));
    c->integer_J = flags[2] == 0;
    // constant row length d (lattices, regular graphs): row i starts at d i, so
    // the lane-per-row kernels need not read the offsets
    if (nnz > 0 && nnz % n == 0) {
        const int64_t d = nnz / n;
        bool regular = true;
        for (int64_t i = 0; i <= n && regular; ++i) regular = rp_host[i] == d * i;
        c->row_len = regular ? static_cast<int32_t>(d) : 0;
    }
    // every value an integer in [-128, 127] (the lattice's +-1 among them):
    // an exact 8-bit copy that the lane-per-row step streams instead; the
    // compact copies are an optimisation, so a device too full to hold
    // them runs without them
    if (nnz > 0 && !flags[3] && dev_alloc(&c->val8, padded) != hipSuccess) {
        c->val8 = nullptr;
        (void)hipGetLastError();
    }
    if (c->val8) {
        if ((e = hipMemsetAsync(c->val8 + nnz, 0, doch::kCsrPad, s)) != hipSuccess) return bail(hip_fail(e, "memset pad"));
        if ((e = doch::launch_csr_pack_i8(csr_view(c), c->val8, s)) != hipSuccess) return bail(hip_fail(e, "pack values"));
        // 4-entry rows (the lattice) whose columns all lie within 32767 of
        // their row, cyclically: the indices as 16-bit offsets too
        if (c->row_len == 4 && !flags[4] && dev_alloc(&c->col16, padded * sizeof(int16_t)) != hipSuccess) {
            c->col16 = nullptr;
            (void)hipGetLastError();
        }
        if (c->col16) {
            if ((e = hipMemsetAsync(c->col16 + nnz, 0, doch::kCsrPad * sizeof(int16_t), s)) != hipSuccess)
                return bail(hip_fail(e, "memset pad"));
            if ((e = doch::launch_csr_pack_col16(csr_view(c), c->col16, s)) != hipSuccess)
                return bail(hip_fail(e, "pack columns"));
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "sync"));
    }
    c->rp_host = std::move(rp_host);
    c->geometry = default_geometry(n, nnz);
    c->wg_per_cu = default_wg_per_cu(c->geometry, c->row_len, c->col16 != nullptr);
    doch::CsrPlan* plan = nullptr;
    if (c->geometry != doch::kGeometryResident && (st = ensure_plan(c, c->geometry, &plan)) != ISING_OK)
        return bail(st);
    *out = c;
    return ISING_OK;
}

ising_status ising_create_dense(int64_t n, const void* J_dev, int32_t jt, int64_t ld,
                                const void* h_dev, int32_t ht, void* stream, ising_ctx** out) {
    if (!out) return fail(ISING_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 1000000) return fail(ISING_E_INVALID_ARG, "n=%lld out of range", (long long)n);
    if (ld < n) return fail(ISING_E_INVALID_ARG, "ld < n");
    if (!J_dev) return fail(ISING_E_INVALID_ARG, "J is NULL");
    if (jt != ISING_F64) return fail(ISING_E_UNSUPPORTED, "dense J must be ISING_F64");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ising_ctx* c = new ising_ctx();
    ising_status st = ISING_OK;
    auto bail = [&](ising_status e) { free_ctx(c); return e; };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(ISING_E_HIP, "no HIP device"));
    c->dense = true;
    c->n = n;
    c->np = n;
    c->nnz = n * (n - 1);
    c->vt = ISING_F64;
    c->ld = n;
    hipError_t e;
    if ((e = dev_alloc(&c->J, static_cast<size_t>(n) * n * sizeof(double))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc(J)"));
    if ((e = hipMemcpy2DAsync(c->J, n * sizeof(double), J_dev, ld * sizeof(double), n * sizeof(double), n,
                              hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return bail(hip_fail(e, "copy J"));
    if ((st = copy_field(c, h_dev, ht, s)) != ISING_OK) return bail(st);
    Scratch sc;
    if ((st = ensure_scratch(c, 0, &sc)) != ISING_OK) return bail(st);
    if ((e = hipMemsetAsync(sc.flags, 0, 8 * sizeof(int32_t), s)) != hipSuccess) return bail(hip_fail(e, "memset"));
    if ((e = doch::launch_dense_validate(dense_view(c), sc.flags, s)) != hipSuccess) return bail(hip_fail(e, "validate"));
    int32_t flags[8];
    if ((e = hipMemcpyAsync(flags, sc.flags, sizeof(flags), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return bail(hip_fail(e, "copy flags"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "sync"));
    if (flags[0]) return bail(fail(ISING_E_INVALID_ARG, "J has a non-finite entry"));
    if (flags[1]) return bail(fail(ISING_E_NONZERO_DIAG, "a diagonal coupling J_ii is nonzero"));
    c->integer_J = flags[2] == 0;
    *out = c;
    return ISING_OK;
}

ising_status ising_create_procedural(int64_t n, int32_t kind, double seed, void* stream,
                                     ising_ctx** out) {
    if (!out) return fail(ISING_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 2 || n > 90000000LL) return fail(ISING_E_INVALID_ARG, "n=%lld out of range", (long long)n);
    if (kind != 1) return fail(ISING_E_INVALID_ARG, "unknown procedural kind %d", kind);
    if (!std::isfinite(seed)) return fail(ISING_E_INVALID_ARG, "seed must be finite");
    // The kernels advance the angle i*j + seed by exact steps and restart from
    // exact integer arguments; both are exact only when every argument is an
    // integer below 2^53 in magnitude.
    if (seed != std::floor(seed))
        return fail(ISING_E_INVALID_ARG, "seed %.17g is not an integer", seed);
    const double nm1 = static_cast<double>(n - 1);
    if (std::fabs(seed) + nm1 * nm1 >= 9007199254740992.0)
        return fail(ISING_E_INVALID_ARG, "|seed| + (n-1)^2 must stay below 2^53");
    (void)stream;
    ising_ctx* c = new ising_ctx();
    if (hipGetDevice(&c->device) != hipSuccess) { free_ctx(c); return fail(ISING_E_HIP, "no HIP device"); }
    c->dense = true;
    c->n = n;
    c->np = n;
    c->nnz = n * (n - 1);
    c->vt = ISING_F64;
    c->ld = n;
    c->proc_kind = kind;
    c->proc_seed = seed;
    c->integer_J = false;
    *out = c;
    return ISING_OK;
}

void ising_destroy(ising_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_ctx(ctx);
}

ising_status ising_get_info(const ising_ctx* ctx, ising_info* out) {
    if (!ctx || !out) return fail(ISING_E_INVALID_ARG, "NULL argument");
    out->n = ctx->n;
    out->n_iter = ctx->np;
    out->nnz = ctx->nnz;
    out->is_dense = ctx->dense ? 1 : 0;
    out->has_field = ctx->has_field ? 1 : 0;
    out->integer_J = ctx->integer_J ? 1 : 0;
    out->val_dtype = ctx->vt;
    out->row_len = ctx->row_len;
    out->geometry = ctx->batch ? -1 : ctx->geometry;
    out->step_val_bytes = ctx->val8 ? 1 : static_cast<int32_t>(ctx->dense ? 8 : dtype_size(ctx->vt));
    out->step_col_bytes = ctx->col16 ? 2 : (ctx->dense ? 0 : 4);
    return ISING_OK;
}

ising_status ising_check_symmetric(ising_ctx* ctx, void* stream) {
    if (!ctx) return fail(ISING_E_INVALID_ARG, "ctx is NULL");
    if (ctx->proc_kind != 0) return ISING_OK;          // sin(i j + seed) is symmetric by construction
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Scratch sc;
    ising_status st = ensure_scratch(ctx, 0, &sc);
    if (st != ISING_OK) return st;
    HIP_OK(hipMemsetAsync(sc.flags, 0, sizeof(int32_t), s), "memset");
    if (ctx->dense) HIP_OK(doch::launch_dense_symcheck(dense_view(ctx), sc.flags, s), "symcheck");
    else HIP_OK(doch::launch_csr_symcheck(csr_view(ctx), sc.flags, s), "symcheck");
    int32_t bad = 0;
    HIP_OK(hipMemcpyAsync(&bad, sc.flags, sizeof(bad), hipMemcpyDeviceToHost, s), "copy");
    HIP_OK(hipStreamSynchronize(s), "sync");
    return bad ? fail(ISING_E_NOT_SYMMETRIC, "J != J^T") : ISING_OK;
}

ising_status ising_default_params(ising_ctx* ctx, double eta, int32_t method, void* stream,
                                  ising_params* out, double* lambda_out) {
    if (!ctx || !out) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(ISING_E_INVALID_ARG, "eta must be > 0");
    if (method < 0 || method > 2) return fail(ISING_E_INVALID_ARG, "method must be 0, 1 or 2");
    if (ctx->np < 2) return fail(ISING_E_INVALID_ARG, "parameter setting needs n' >= 2");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = 1024;
    Scratch sc;
    ising_status st = ensure_scratch(ctx, static_cast<size_t>(2048) * 4, &sc);
    if (st != ISING_OK) return st;
    HIP_OK(hipMemsetAsync(sc.tickets, 0, sizeof(unsigned int), s), "memset");
    // pass 0: row sums, sum, count; pass 1: squared deviations from the mean
    const double np = static_cast<double>(ctx->np);
    const double m = np * (np - 1.0);
    MatrixStats ms;
    for (int pass = 0; pass < 2; ++pass) {
        const double mean = pass == 0 ? 0.0 : ms.s1 / m;
        if (ctx->dense)
            HIP_OK(doch::launch_dense_stats(dense_view(ctx), mean, pass, sc.partials, sc.tickets, grid, sc.stats, s), "stats");
        else
            HIP_OK(doch::launch_csr_stats(csr_view(ctx), mean, pass, sc.partials, sc.tickets, grid, sc.stats, s), "stats");
        HIP_OK(hipMemcpyAsync(&ms, sc.stats, sizeof(ms), hipMemcpyDeviceToHost, s), "copy stats");
        HIP_OK(hipStreamSynchronize(s), "sync");
    }
    const double jbar = ms.s1 / m;
    // entries not stored are zeros: each adds (0 - jbar)^2
    const double ss = ms.ss + (m - ms.stored) * jbar * jbar;
    const double wigner = 2.0 * std::sqrt(ss / m) * std::sqrt(np);
    double lambda = wigner;
    const bool power = method == 1 || (method == 0 && ctx->np < 10000);
    if (power) {
        // power iteration on c I - Jhat from a fixed pseudo-random start
        const double c = ms.abs_max;
        const int64_t nv = ctx->np;
        std::vector<double> v0(static_cast<size_t>(nv));
        uint64_t z = 0x9E3779B97F4A7C15ULL;
        double nrm = 0.0;
        for (int64_t i = 0; i < nv; ++i) {
            z += 0x9E3779B97F4A7C15ULL;   // SplitMix64 (Steele, Lea, Flood 2014)
            uint64_t q = z;
            q = (q ^ (q >> 30)) * 0xBF58476D1CE4E5B9ULL;
            q = (q ^ (q >> 27)) * 0x94D049BB133111EBULL;
            q ^= q >> 31;
            v0[i] = 2.0 * (static_cast<double>(q >> 11) * 0x1.0p-53) - 1.0;
            nrm += v0[i] * v0[i];
        }
        nrm = std::sqrt(nrm);
        for (auto& x : v0) x /= nrm;
        double* v = sc.vecs;
        double* w = sc.vecs + nv;
        HIP_OK(hipMemcpyAsync(v, v0.data(), nv * sizeof(double), hipMemcpyHostToDevice, s), "copy v0");
        const int64_t maxit = 100000;
        const double tol = 1e-12;
        double mu = 0.0, mu_prev = 0.0;
        bool conv = false;
        std::vector<double> mlog(2 * kPowerChunk);
        for (int64_t k0 = 0; k0 < maxit && !conv; k0 += kPowerChunk) {
            const int64_t cnt = std::min<int64_t>(kPowerChunk, maxit - k0);
            for (int64_t j = 0; j < cnt; ++j) {
                if (ctx->dense)
                    HIP_OK(doch::launch_dense_power_step(dense_view(ctx), c, v, w, sc.partials, sc.tickets,
                                                         doch::dense_step_grid(ctx->n), sc.mu_log, j, s), "power");
                else
                    HIP_OK(doch::launch_csr_power_step(csr_view(ctx), c, v, w, sc.partials, sc.tickets, grid,
                                                       sc.mu_log, j, s), "power");
                HIP_OK(doch::launch_normalize(w, v, sc.mu_log, j, nv, s), "normalize");
            }
            HIP_OK(hipMemcpyAsync(mlog.data(), sc.mu_log, 2 * cnt * sizeof(double), hipMemcpyDeviceToHost, s),
                   "copy mu");
            HIP_OK(hipStreamSynchronize(s), "sync");
            for (int64_t j = 0; j < cnt; ++j) {
                mu = mlog[2 * j];
                if (!std::isfinite(mu)) return fail(ISING_E_NONFINITE, "power iteration diverged");
                if ((k0 + j) > 0 && std::fabs(mu - mu_prev) <= tol * std::fabs(mu)) {
                    conv = true;
                    break;
                }
                mu_prev = mu;
                if (mlog[2 * j + 1] == 0.0) { conv = true; break; }
            }
        }
        lambda = mu - c;
    }
    ctx->last_lambda = lambda;
    ctx->last_rowsum = ms.rowsum_max;
    ising_params p;
    p.alpha = eta * lambda;
    p.beta = std::pow(np, 1.5) * (p.alpha + ms.rowsum_max);
    p.eps = 0.0;
    p.algo = 0;
    p.q = 5;
    p.x_dtype = ISING_F64;
    p.reserved = 0;
    *out = p;
    if (lambda_out) *lambda_out = lambda;
    return ISING_OK;
}

ising_status ising_solve(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t iters,
                         const ising_params* params, double* x_out_dev, int8_t* s_out_dev,
                         ising_stats* stats_host, void* stream) {
    if (!ctx || !params) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (!x0_dev) return fail(ISING_E_INVALID_ARG, "x0 is NULL");
    if (R < 1 || R > kMaxR) return fail(ISING_E_INVALID_ARG, "R=%d out of range", R);
    if (iters < 0) return fail(ISING_E_INVALID_ARG, "iters < 0");
    const ising_params& p = *params;
    if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return fail(ISING_E_INVALID_ARG, "alpha must be finite and > 0");
    if (!(p.beta > 0.0) || !std::isfinite(p.beta)) return fail(ISING_E_INVALID_ARG, "beta must be finite and > 0");
    if (!(p.eps >= 0.0)) return fail(ISING_E_INVALID_ARG, "eps must be >= 0");
    if (p.x_dtype != ISING_F64 && p.x_dtype != ISING_F32) return fail(ISING_E_INVALID_ARG, "x_dtype must be F64 or F32");
    if (p.reserved != 0) return fail(ISING_E_INVALID_ARG, "reserved must be 0");
    if (p.algo != 0 && p.algo != 1) return fail(ISING_E_INVALID_ARG, "algo must be 0 or 1");
    if (p.algo == 1) {
        if (ctx->batch) return fail(ISING_E_UNSUPPORTED, "ADOCH runs on single CSR or dense contexts");
        if (R != 1 && R != 2 && R != 4 && R != 8)
            return fail(ISING_E_UNSUPPORTED, "ADOCH runs 1, 2, 4 or 8 restarts together");
        if (p.x_dtype != ISING_F64) return fail(ISING_E_UNSUPPORTED, "ADOCH stores its iterates in FP64");
        if (p.q < 1) return fail(ISING_E_INVALID_ARG, "ADOCH needs q >= 1");
        return solve_adoch(ctx, x0_dev, R, iters, p, x_out_dev, s_out_dev, stats_host,
                           static_cast<hipStream_t>(stream));
    }
    if (ctx->batch) return fail(ISING_E_UNSUPPORTED, "use ising_solve_batch on a batch context");
    if (R != 1) return fail(ISING_E_UNSUPPORTED, "R > 1: use ising_solve_batch or ising_solve_lowp");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (resident_selected(ctx))
        return solve_resident(ctx, x0_dev, iters, p, x_out_dev, s_out_dev, stats_host, s);
    const size_t elt = p.x_dtype == ISING_F64 ? 8 : 4;
    const size_t xbytes = static_cast<size_t>(ctx->np) * R * elt;
    if (!ctx->xbuf[0] || ctx->xbuf_bytes < xbytes) {
        dev_free(ctx->xbuf[0]);
        dev_free(ctx->xbuf[1]);
        ctx->xbuf_bytes = 0;
        HIP_OK(dev_alloc(&ctx->xbuf[0], xbytes), "hipMalloc(x)");
        HIP_OK(dev_alloc(&ctx->xbuf[1], xbytes), "hipMalloc(x)");
        ctx->xbuf_bytes = xbytes;
    }
    doch::CsrPlan* plan = nullptr;
    if (!ctx->dense) {
        ising_status pst = ensure_plan(ctx, ctx->geometry, &plan);
        if (pst != ISING_OK) return pst;
        plan->wg_per_cu = ctx->wg_per_cu;
    }
    // upper bound of the step kernels' grids: every workgroup that can be
    // resident at once (256 CUs x at most 8 workgroups of 256 threads)
    const int grid = ctx->dense ? doch::dense_step_grid(ctx->n) : 0;
    const size_t max_grid = ctx->dense ? static_cast<size_t>(grid) : static_cast<size_t>(doch::kMaxStepGrid);
    HIP_OK(ensure(&ctx->partials, &ctx->partials_bytes,
                  max_grid * R * doch::kNumPartials * sizeof(double)), "hipMalloc(partials)");
    ising_status sst = ensure_solve_state(ctx, iters, R);
    if (sst != ISING_OK) return sst;
    unsigned int* sched = ctx->ticket + kMaxR;
    HIP_OK(doch::launch_init_state(ctx->state, R, ctx->ticket, sched, s), "init");
    HIP_OK(doch::launch_load_x0(x0_dev, ctx->xbuf[0], p.x_dtype, ctx->np * R, s), "load x0");
    StepArgs a;
    a.x_dtype = p.x_dtype;
    a.R = R;
    a.alpha = p.alpha;
    a.beta = p.beta;
    a.eps = p.eps;
    a.partials = ctx->partials;
    a.ticket = ctx->ticket;
    a.sched = ctx->dense ? nullptr : sched;
    a.state = ctx->state;
    a.all_done_flag = 0;
    const CsrView cv = csr_view(ctx);
    const DenseView dv = dense_view(ctx);
    for (int64_t k = 0; k < iters; ++k) {
        a.x_old = ctx->xbuf[k & 1];
        a.x_new = ctx->xbuf[(k + 1) & 1];
        a.k = k;
        a.log = ctx->log;
        hipError_t e = ctx->dense ? doch::launch_dense_step(dv, a, grid, s)
                                  : doch::launch_csr_step(cv, *plan, a, s);
        if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    ctx->last_R = R;
    ctx->last_iters = iters;
    ctx->last_adoch = false;
    if (x_out_dev || s_out_dev)
        HIP_OK(doch::launch_finish(ctx->xbuf[0], ctx->xbuf[1], nullptr, p.x_dtype, ctx->state, ctx->n, ctx->np, R,
                                   ctx->has_field, x_out_dev, s_out_dev, s), "finish");
    return read_stats(ctx, R, stats_host, s);
}

ising_status ising_set_geometry(ising_ctx* ctx, int32_t geometry, int32_t wg_per_cu) {
    if (!ctx) return fail(ISING_E_INVALID_ARG, "ctx is NULL");
    if (ctx->batch) return fail(ISING_E_UNSUPPORTED, "geometries apply to single CSR or dense contexts");
    if (wg_per_cu < 0 || wg_per_cu > 32) return fail(ISING_E_INVALID_ARG, "wg_per_cu out of range");
    if (ctx->dense) {
        if (geometry != -1 && geometry != 0 && geometry != doch::kGeometryResident)
            return fail(ISING_E_INVALID_ARG, "dense contexts take geometry -1, 0 or %d", doch::kGeometryResident);
        if (geometry == doch::kGeometryResident && (ctx->proc_kind != 0 || ctx->n > doch::kResidentMaxDense))
            return fail(ISING_E_UNSUPPORTED, "the resident solve holds stored dense matrices of order <= %lld",
                        (long long)doch::kResidentMaxDense);
        ctx->geometry = geometry;
        return ISING_OK;
    }
    if (geometry < -1 || geometry > doch::kGeometryResident) return fail(ISING_E_INVALID_ARG, "bad geometry");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    const int g = geometry < 0 ? default_geometry(ctx->n, ctx->nnz) : geometry;
    if (g != doch::kGeometryResident) {
        doch::CsrPlan* plan = nullptr;
        ising_status st = ensure_plan(ctx, g, &plan);
        if (st != ISING_OK) return st;
    }
    ctx->geometry = g;
    ctx->wg_per_cu = geometry < 0 ? default_wg_per_cu(g, ctx->row_len, ctx->col16 != nullptr) : wg_per_cu;
    return ISING_OK;
}

ising_status ising_autotune(ising_ctx* ctx, const double* x0_dev, int64_t iters,
                            const ising_params* params, void* stream, int32_t* geometry_out,
                            int32_t* wg_per_cu_out, double* ms_per_iter_out) {
    if (!ctx || !params || !x0_dev) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (ctx->dense || ctx->batch) return fail(ISING_E_UNSUPPORTED, "geometries are tuned on single CSR contexts");
    if (iters < 1) return fail(ISING_E_INVALID_ARG, "iters < 1");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0), "event");
    HIP_OK(hipEventCreate(&e1), "event");
    int best = -1, best_wpc = 0;
    float best_ms = 0.0f;
    ising_params p = *params;
    p.eps = 0.0;                     // time exactly `iters` iterations
    ising_status st = ISING_OK;
    // workgroups per CU to try (0 = as many as fit); the resident solve has
    // a single launch shape
    const int wpcs[] = {1, 2, 3, 4, 0};
    for (int g = 0; g <= doch::kGeometryResident && st == ISING_OK; ++g) {
        float g_best = 0.0f;
        for (int w : wpcs) {
            if (g == doch::kGeometryResident && (w != 0 || ctx->n > kResidentTuneMaxRows)) continue;
            if ((st = ising_set_geometry(ctx, g, w)) != ISING_OK) break;
            if ((st = ising_solve(ctx, x0_dev, 1, 1, &p, nullptr, nullptr, nullptr, stream)) != ISING_OK) break;
            // best of two timings of `iters` iterations
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && st == ISING_OK; ++rep) {
                if (hipEventRecord(e0, s) != hipSuccess) { st = fail(ISING_E_HIP, "event record"); break; }
                if ((st = ising_solve(ctx, x0_dev, 1, iters, &p, nullptr, nullptr, nullptr, stream)) != ISING_OK) break;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = fail(ISING_E_HIP, "event sync");
                    break;
                }
                float t = 0.0f;
                (void)hipEventElapsedTime(&t, e0, e1);
                if (rep == 0 || t < ms) ms = t;
            }
            if (st != ISING_OK) break;
            if (g_best == 0.0f || ms < g_best) g_best = ms;
            if (best < 0 || ms < best_ms) { best = g; best_wpc = w; best_ms = ms; }
        }
        if (ms_per_iter_out) ms_per_iter_out[g] = g_best / static_cast<double>(iters);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ISING_OK) return st;
    ctx->geometry = best;
    ctx->wg_per_cu = best_wpc;
    if (geometry_out) *geometry_out = best;
    if (wg_per_cu_out) *wg_per_cu_out = best_wpc;
    return ISING_OK;
}

namespace {

BatchView batch_view(const ising_ctx* c) {
    BatchView b;
    b.count = c->count;
    b.rp = c->rp;
    b.col = c->col;
    b.val = c->val;
    b.vt = c->vt;
    b.inst = c->inst;
    b.order = c->order;
    return b;
}

}  // namespace

ising_status ising_create_batch(int32_t count, const int64_t* n_host, const int32_t* row_ptr_dev,
                                const int32_t* col_dev, const void* val_dev, int32_t vt,
                                void* stream, ising_ctx** out) {
    if (!out) return fail(ISING_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !n_host) return fail(ISING_E_INVALID_ARG, "count < 1 or n is NULL");
    int64_t total = 0;
    for (int32_t k = 0; k < count; ++k) {
        if (n_host[k] < 2) return fail(ISING_E_INVALID_ARG, "instance %d has n < 2", k);
        total += n_host[k];
    }
    if (total >= 2147483647LL) return fail(ISING_E_INVALID_ARG, "total rows out of range");
    if (!row_ptr_dev) return fail(ISING_E_INVALID_ARG, "row_ptr is NULL");
    if (!float_dtype(vt)) return fail(ISING_E_INVALID_ARG, "batch values must be ISING_F32 or ISING_F64");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t nnz32 = 0;
    HIP_OK(hipMemcpyAsync(&nnz32, row_ptr_dev + total, sizeof(int32_t), hipMemcpyDeviceToHost, s), "read nnz");
    HIP_OK(hipStreamSynchronize(s), "sync");
    ising_ctx* c = nullptr;
    ising_status st = ising_create_csr(total, nnz32, row_ptr_dev, col_dev, val_dev, vt, nullptr, ISING_F32,
                                       stream, &c);
    if (st != ISING_OK) return st;
    auto bail = [&](ising_status e) { free_ctx(c); return e; };
    c->batch = true;
    c->count = count;
    c->inst_host.resize(static_cast<size_t>(count));
    int64_t row = 0;
    for (int32_t k = 0; k < count; ++k) {
        BatchInstance& I = c->inst_host[k];
        I.row0 = static_cast<int32_t>(row);
        I.n = static_cast<int32_t>(n_host[k]);
        I.e0 = c->rp_host[row];
        I.nnz = c->rp_host[row + n_host[k]] - I.e0;
        row += n_host[k];
    }
    // largest instances first
    std::vector<int32_t> order(static_cast<size_t>(count));
    for (int32_t k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int64_t wa = static_cast<int64_t>(c->inst_host[a].nnz) + c->inst_host[a].n;
        const int64_t wb = static_cast<int64_t>(c->inst_host[b].nnz) + c->inst_host[b].n;
        return wa > wb;
    });
    hipError_t e;
    if ((e = dev_alloc(&c->inst, count * sizeof(BatchInstance))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(inst)"));
    if ((e = dev_alloc(&c->order, count * sizeof(int32_t))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(order)"));
    if ((e = dev_alloc(&c->bparams, 2 * count * sizeof(double))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(params)"));
    if ((e = dev_alloc(&c->bclock, (count + 1) * sizeof(uint64_t))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(clock)"));
    if ((e = dev_alloc(&c->bqueue, 256)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(queue)"));
    if ((e = hipMemcpy(c->inst, c->inst_host.data(), count * sizeof(BatchInstance), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "copy inst"));
    if ((e = hipMemcpy(c->order, order.data(), count * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "copy order"));
    Scratch sc;
    if ((st = ensure_scratch(c, 0, &sc)) != ISING_OK) return bail(st);
    if ((e = hipMemsetAsync(sc.flags, 0, sizeof(int32_t), s)) != hipSuccess) return bail(hip_fail(e, "memset"));
    if ((e = doch::launch_batch_validate(batch_view(c), total, sc.flags, s)) != hipSuccess)
        return bail(hip_fail(e, "validate blocks"));
    int32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, sc.flags, sizeof(bad), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return bail(hip_fail(e, "copy flag"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "sync"));
    if (bad) return bail(fail(ISING_E_INVALID_ARG, "a coupling leaves its instance's diagonal block"));
    *out = c;
    return ISING_OK;
}

ising_status ising_default_params_batch(ising_ctx* ctx, double eta, int32_t method, void* stream,
                                        double* alpha_host, double* beta_host, double* lambda_host) {
    if (!ctx || !ctx->batch) return fail(ISING_E_INVALID_ARG, "not a batch context");
    if (!alpha_host || !beta_host) return fail(ISING_E_INVALID_ARG, "NULL output");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(ISING_E_INVALID_ARG, "eta must be > 0");
    if (method < 0 || method > 2) return fail(ISING_E_INVALID_ARG, "method must be 0, 1 or 2");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int count = ctx->count;
    // scratch: stats[4*count], shift[count], lam[count], jobs[count], v[np], w[np]
    Scratch sc;
    ising_status st = ensure_scratch(ctx, static_cast<size_t>(7) * count + 16, &sc);
    if (st != ISING_OK) return st;
    double* dstats = sc.partials;
    double* dshift = dstats + 4 * count;
    double* dlam = dshift + count;
    int32_t* djobs = reinterpret_cast<int32_t*>(dlam + count);
    HIP_OK(doch::launch_batch_stats(batch_view(ctx), dstats, s), "batch stats");
    std::vector<double> hs(4 * static_cast<size_t>(count));
    HIP_OK(hipMemcpyAsync(hs.data(), dstats, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy stats");
    HIP_OK(hipStreamSynchronize(s), "sync");
    std::vector<double> lam(static_cast<size_t>(count));
    std::vector<int32_t> jobs;
    std::vector<double> shift(static_cast<size_t>(count));
    for (int k = 0; k < count; ++k) {
        const double n = ctx->inst_host[k].n;
        const double m = n * (n - 1.0);
        const double jbar = hs[4 * k + 1] / m;
        const double ss = hs[4 * k + 3] + (m - hs[4 * k + 2]) * jbar * jbar;
        lam[k] = 2.0 * std::sqrt(ss / m) * std::sqrt(n);
        shift[k] = hs[4 * k + 0];
        if (method == 1 || (method == 0 && ctx->inst_host[k].n < 10000)) jobs.push_back(k);
    }
    if (!jobs.empty()) {
        HIP_OK(hipMemcpyAsync(dshift, shift.data(), count * sizeof(double), hipMemcpyHostToDevice, s), "copy shift");
        HIP_OK(hipMemcpyAsync(djobs, jobs.data(), jobs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
               "copy jobs");
        HIP_OK(doch::launch_batch_power(batch_view(ctx), djobs, static_cast<int>(jobs.size()), dshift, 1e-12,
                                        100000, sc.vecs, sc.vecs + ctx->np, dlam, s), "batch power");
        std::vector<double> pl(static_cast<size_t>(count));
        HIP_OK(hipMemcpyAsync(pl.data(), dlam, count * sizeof(double), hipMemcpyDeviceToHost, s), "copy lambda");
        HIP_OK(hipStreamSynchronize(s), "sync");
        for (int32_t k : jobs) lam[k] = pl[k];
    }
    for (int k = 0; k < count; ++k) {
        const double n = ctx->inst_host[k].n;
        alpha_host[k] = eta * lam[k];
        beta_host[k] = std::pow(n, 1.5) * (alpha_host[k] + hs[4 * k + 0]);
        if (lambda_host) lambda_host[k] = lam[k];
    }
    return ISING_OK;
}

// Default launch shape of the batch solve for R <= 8 restarts: every
// restart of an instance in one unit (a row's R iterate entries share one
// cache line, so splitting the restarts multiplies the lines the gathers
// fetch), 256 threads (512 below 4 restarts per unit), chunks of 512 rows.
static doch::BatchShape default_batch_shape(int R) {
    doch::BatchShape sh;
    sh.rj = std::min(8, R);
    sh.wg = sh.rj >= 4 ? 256 : 512;
    sh.chunk_rows = 512;
    return sh;
}

static doch::BatchShape batch_shape_for(const ising_ctx* ctx, int R) {
    if (ctx->bshape_set && doch::batch_shape_supported(ctx->bshape, R)) return ctx->bshape;
    return default_batch_shape(R);
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// The plan of the lockstep batch solve for R <= 8 restarts and shape `sh`:
// units (restart groups of instances) dealt to the XCDs largest first, each
// to the XCD with the least work so far; each unit's rows cut into chunks
// of sh.chunk_rows rows (the last one shorter).
static ising_status ensure_batch_plan(ising_ctx* ctx, int R, const doch::BatchShape& sh, int x_dtype,
                                      hipStream_t s) {
    const std::vector<int64_t> key = {R, sh.rj, sh.wg, sh.chunk_rows, x_dtype};
    if (ctx->bplan_mem && ctx->bplan_key == key) return ISING_OK;
    if (R > 8) {
        ctx->bplan_key = key;
        return ISING_OK;
    }
    const int RJ = std::min(sh.rj, R);
    const int groups = R / RJ;
    int cus = 256;
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device), "CU count");
    const int n_xcd = std::max(1, std::min(doch::kBatchMaxXcd, cus / 32));
    std::vector<int32_t> order(static_cast<size_t>(ctx->count));
    for (int k = 0; k < ctx->count; ++k) order[k] = k;
    auto work = [&](int k) { return static_cast<int64_t>(ctx->inst_host[k].nnz) + ctx->inst_host[k].n; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work(a) > work(b); });
    std::vector<std::vector<int32_t>> bins(static_cast<size_t>(n_xcd));   // units per XCD
    std::vector<int64_t> load(static_cast<size_t>(n_xcd), 0);
    std::vector<doch::BatchUnit> units;
    for (int32_t k : order)
        for (int g = 0; g < groups; ++g) {
            const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
            doch::BatchUnit U;
            U.inst = k;
            U.r0 = g * RJ;
            U.first_slot = 0;
            U.nchunks = 0;
            bins[x].push_back(static_cast<int32_t>(units.size()));
            units.push_back(U);
            load[x] += work(k);
        }
    std::vector<doch::BatchChunk> chunks;
    std::vector<int32_t> off(doch::kBatchMaxXcd + 1, 0), units_on(doch::kBatchMaxXcd, 0);
    for (int x = 0; x < doch::kBatchMaxXcd; ++x) {
        off[x] = static_cast<int32_t>(chunks.size());
        if (x >= n_xcd) continue;
        units_on[x] = static_cast<int32_t>(bins[x].size());
        for (int32_t u : bins[x]) {
            const doch::BatchInstance& I = ctx->inst_host[units[u].inst];
            units[u].first_slot = static_cast<int32_t>(chunks.size());
            for (int lo = 0; lo < I.n; lo += sh.chunk_rows) {
                doch::BatchChunk c;
                c.unit = u;
                c.lo = I.row0 + lo;
                c.hi = I.row0 + std::min(I.n, lo + sh.chunk_rows);
                c.slot = static_cast<int32_t>(chunks.size());
                chunks.push_back(c);
                ++units[u].nchunks;
            }
        }
    }
    off[doch::kBatchMaxXcd] = static_cast<int32_t>(chunks.size());
    const size_t K = 4 * static_cast<size_t>(RJ);
    const size_t nu = units.size();
    const size_t b_args = align256(sizeof(doch::BatchStepArgs));
    const size_t b_units = align256(nu * sizeof(doch::BatchUnit));
    const size_t b_chunks = align256(chunks.size() * sizeof(doch::BatchChunk));
    const size_t b_off = align256(off.size() * sizeof(int32_t));
    const size_t b_on = align256(units_on.size() * sizeof(int32_t));
    const size_t b_counters = align256(doch::kBatchCounterWords * sizeof(unsigned int));
    const size_t b_tickets = align256(nu * 32 * sizeof(unsigned int));
    const size_t b_done = align256(nu * sizeof(int32_t));
    const size_t b_conv = align256(nu * RJ * sizeof(int32_t));
    const size_t b_partials = align256(chunks.size() * K * sizeof(double));
    const size_t total =
        b_args + b_units + b_chunks + b_off + b_on + b_counters + b_tickets + b_done + b_conv + b_partials;
    HIP_OK(ensure(&ctx->bplan_mem, &ctx->bplan_bytes, total), "hipMalloc(batch plan)");
    char* p = static_cast<char*>(ctx->bplan_mem);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += bytes;
        return q;
    };
    ctx->bargs_dev = reinterpret_cast<doch::BatchStepArgs*>(take(b_args));
    auto* d_units = reinterpret_cast<doch::BatchUnit*>(take(b_units));
    auto* d_chunks = reinterpret_cast<doch::BatchChunk*>(take(b_chunks));
    auto* d_off = reinterpret_cast<int32_t*>(take(b_off));
    auto* d_on = reinterpret_cast<int32_t*>(take(b_on));
    doch::BatchPlan& pl = ctx->bplan;
    pl.units = d_units;
    pl.chunks = d_chunks;
    pl.off = d_off;
    pl.units_on = d_on;
    pl.counters = reinterpret_cast<unsigned int*>(take(b_counters));
    pl.tickets = reinterpret_cast<unsigned int*>(take(b_tickets));
    pl.done = reinterpret_cast<int32_t*>(take(b_done));
    pl.conv = reinterpret_cast<int32_t*>(take(b_conv));
    pl.partials = reinterpret_cast<double*>(take(b_partials));
    pl.n_units = static_cast<int32_t>(nu);
    pl.n_slots = static_cast<int32_t>(chunks.size());
    pl.n_xcd = n_xcd;
    pl.rj = RJ;
    HIP_OK(hipMemcpyAsync(d_units, units.data(), nu * sizeof(doch::BatchUnit), hipMemcpyHostToDevice, s), "copy units");
    HIP_OK(hipMemcpyAsync(d_chunks, chunks.data(), chunks.size() * sizeof(doch::BatchChunk), hipMemcpyHostToDevice, s),
           "copy chunks");
    HIP_OK(hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy offsets");
    HIP_OK(hipMemcpyAsync(d_on, units_on.data(), units_on.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
           "copy unit counts");
    HIP_OK(hipStreamSynchronize(s), "sync");
    ctx->bplan_key = key;
    return ISING_OK;
}

ising_status ising_solve_batch(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t max_iters,
                               const double* alpha_host, const double* beta_host, double eps,
                               int32_t x_dtype, double* x_out_dev, int8_t* s_out_dev,
                               ising_stats* stats_host, double* tts_ms_host, void* stream) {
    if (!ctx || !ctx->batch) return fail(ISING_E_INVALID_ARG, "not a batch context");
    if (!x0_dev || !alpha_host || !beta_host) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (!doch::batch_restarts_supported(R)) return fail(ISING_E_INVALID_ARG, "R must be 1, 2, 4, 8, 16 or 32");
    if (max_iters < 0) return fail(ISING_E_INVALID_ARG, "max_iters < 0");
    if (!(eps >= 0.0)) return fail(ISING_E_INVALID_ARG, "eps must be >= 0");
    if (x_dtype != ISING_F64 && x_dtype != ISING_F32) return fail(ISING_E_INVALID_ARG, "x_dtype must be F64 or F32");
    const int count = ctx->count;
    for (int k = 0; k < count; ++k)
        if (!(alpha_host[k] > 0.0) || !(beta_host[k] > 0.0) || !std::isfinite(alpha_host[k]) ||
            !std::isfinite(beta_host[k]))
            return fail(ISING_E_INVALID_ARG, "instance %d: alpha and beta must be finite and > 0", k);
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t elt = x_dtype == ISING_F64 ? 8 : 4;
    const size_t xbytes = static_cast<size_t>(ctx->np) * R * elt;
    if (!ctx->xbuf[0] || ctx->xbuf_bytes < xbytes) {
        dev_free(ctx->xbuf[0]);
        dev_free(ctx->xbuf[1]);
        ctx->xbuf_bytes = 0;
        HIP_OK(dev_alloc(&ctx->xbuf[0], xbytes), "hipMalloc(x)");
        HIP_OK(dev_alloc(&ctx->xbuf[1], xbytes), "hipMalloc(x)");
        ctx->xbuf_bytes = xbytes;
    }
    HIP_OK(ensure(&ctx->bstats, &ctx->bstats_bytes, static_cast<size_t>(count) * R * sizeof(BatchRestartStat)),
           "hipMalloc(stats)");
    std::vector<double> ab(2 * static_cast<size_t>(count));
    std::copy(alpha_host, alpha_host + count, ab.begin());
    std::copy(beta_host, beta_host + count, ab.begin() + count);
    HIP_OK(hipMemcpyAsync(ctx->bparams, ab.data(), ab.size() * sizeof(double), hipMemcpyHostToDevice, s),
           "copy alpha/beta");
    const doch::BatchShape shape = batch_shape_for(ctx, R);
    ising_status pst = ensure_batch_plan(ctx, R, shape, x_dtype, s);
    if (pst != ISING_OK) return pst;
    // the whole solve is one persistent kernel (after a small init kernel),
    // captured once into a graph and replayed while the arguments repeat
    const std::vector<uint64_t> key = {static_cast<uint64_t>(R), static_cast<uint64_t>(shape.rj),
                                       static_cast<uint64_t>(shape.wg), static_cast<uint64_t>(shape.chunk_rows),
                                       reinterpret_cast<uint64_t>(ctx->bplan_mem),
                                       static_cast<uint64_t>(max_iters),
                                       static_cast<uint64_t>(x_dtype), reinterpret_cast<uint64_t>(x0_dev),
                                       reinterpret_cast<uint64_t>(x_out_dev), reinterpret_cast<uint64_t>(s_out_dev),
                                       reinterpret_cast<uint64_t>(ctx->xbuf[0]), reinterpret_cast<uint64_t>(ctx->bstats),
                                       reinterpret_cast<uint64_t>(s), static_cast<uint64_t>(std::hash<double>{}(eps))};
    if (!ctx->bgraph || ctx->bgraph_key != key) {
        if (ctx->bgraph) { (void)hipGraphExecDestroy(ctx->bgraph); ctx->bgraph = nullptr; }
        if (ctx->bgraph_src) { (void)hipGraphDestroy(ctx->bgraph_src); ctx->bgraph_src = nullptr; }
        if (R <= 8) {
            // the kernel's arguments, in stream order after earlier solves
            doch::BatchStepArgs& ta = ctx->bargs_host;
            ta.inst = ctx->inst;
            ta.R = R;
            ta.alpha = ctx->bparams;
            ta.beta = ctx->bparams + count;
            ta.eps = eps;
            ta.max_iters = max_iters;
            ta.x0 = x0_dev;
            ta.plan = ctx->bplan;
            ta.stats = ctx->bstats;
            ta.clock_start = ctx->bclock;
            ta.clock_end = ctx->bclock + 1;
            ta.x_out = x_out_dev;
            ta.s_out = s_out_dev;
            HIP_OK(hipMemcpyAsync(ctx->bargs_dev, &ta, sizeof(ta), hipMemcpyHostToDevice, s), "copy batch arguments");
        }
        hipStream_t cs;
        HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            e = doch::launch_batch_solve(batch_view(ctx), R, shape, ctx->bplan, ctx->bargs_dev, max_iters,
                                         ctx->bparams,
                                         ctx->bparams + count, eps,
                                         x_dtype, x0_dev, ctx->xbuf[0], ctx->xbuf[1], ctx->bqueue, ctx->bstats,
                                         ctx->bclock, ctx->bclock + 1, x_out_dev, s_out_dev, cs);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&ctx->bgraph, g, nullptr, nullptr, 0);
            if (e == hipSuccess) ctx->bgraph_src = g;
            else if (g) (void)hipGraphDestroy(g);
        }
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            ctx->bgraph = nullptr;
            return hip_fail(e, "batch graph capture");
        }
        ctx->bgraph_key = key;
    }
    HIP_OK(hipGraphLaunch(ctx->bgraph, s), "batch graph launch");
    if (stats_host || tts_ms_host) {
        std::vector<BatchRestartStat> hs(static_cast<size_t>(count) * R);
        std::vector<uint64_t> clk(static_cast<size_t>(count) + 1);
        HIP_OK(hipMemcpyAsync(hs.data(), ctx->bstats, hs.size() * sizeof(BatchRestartStat), hipMemcpyDeviceToHost, s),
               "copy stats");
        HIP_OK(hipMemcpyAsync(clk.data(), ctx->bclock, clk.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s),
               "copy clocks");
        unsigned int aborted = 0;
        if (R <= 8)
            HIP_OK(hipMemcpyAsync(&aborted, ctx->bplan.counters + 32 * 25, sizeof(aborted), hipMemcpyDeviceToHost, s),
                   "copy abort word");
        HIP_OK(hipStreamSynchronize(s), "sync");
        if (aborted) return fail(ISING_E_HIP, "the batch kernel's workgroups timed out waiting at a barrier");
        if (max_iters > 0)
            for (size_t q = 0; q < hs.size(); ++q)
                if (hs[q].iters_done < 1)
                    return fail(ISING_E_HIP, "restart %zu of the batch was never run", q);
        bool bad = false;
        if (stats_host) {
            for (size_t q = 0; q < hs.size(); ++q) {
                stats_host[q].iters_done = hs[q].iters_done;
                stats_host[q].converged = hs[q].converged;
                stats_host[q].nonfinite = hs[q].nonfinite;
                stats_host[q].H_last = hs[q].H_last;
                stats_host[q].r_last = hs[q].r_last;
                bad = bad || hs[q].nonfinite;
            }
        }
        if (tts_ms_host) {
            int rate_khz = 0;
            HIP_OK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device), "clock rate");
            const double ms_per_tick = rate_khz > 0 ? 1.0 / rate_khz : 1e-5;
            for (int k = 0; k < count; ++k)
                tts_ms_host[k] = static_cast<double>(clk[1 + k] - clk[0]) * ms_per_tick;
        }
        if (bad) return fail(ISING_E_NONFINITE, "H or r became non-finite");
    }
    return ISING_OK;
}

ising_status ising_energy_batch(ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* E_dev,
                                int64_t* E_int_dev, void* stream) {
    if (!ctx || !ctx->batch) return fail(ISING_E_INVALID_ARG, "not a batch context");
    if (!s_dev) return fail(ISING_E_INVALID_ARG, "s is NULL");
    if (!doch::batch_restarts_supported(R)) return fail(ISING_E_INVALID_ARG, "R must be 1, 2, 4, 8, 16 or 32");
    if (!E_dev && !E_int_dev) return fail(ISING_E_INVALID_ARG, "no output requested");
    if (E_int_dev && !ctx->integer_J) return fail(ISING_E_UNSUPPORTED, "integer energy needs integer couplings");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_OK(doch::launch_batch_energy(batch_view(ctx), s_dev, R, E_dev, E_int_dev, static_cast<hipStream_t>(stream)),
           "batch energy");
    return ISING_OK;
}

ising_status ising_autotune_lowp(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t iters,
                                 const ising_params* params, int32_t jx_dtype, const char* cache_path, void* stream,
                                 int32_t* shape_out, double* ms_out, int32_t* from_cache_out) {
    if (!ctx || !params || !x0_dev) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (!ctx->dense || ctx->proc_kind != 0)
        return fail(ISING_E_UNSUPPORTED, "the low-precision path needs a stored dense context");
    if (jx_dtype != ISING_BF16 && jx_dtype != ISING_FP8_E4M3)
        return fail(ISING_E_INVALID_ARG, "jx_dtype must be ISING_BF16 or ISING_FP8_E4M3");
    if (R < 1 || R > kMaxR) return fail(ISING_E_INVALID_ARG, "R=%d out of range", R);
    if (iters < 1) return fail(ISING_E_INVALID_ARG, "iters < 1");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, ctx->device), "device properties");
    const int prec = jx_dtype == ISING_BF16 ? 0 : 1;
    const int n = static_cast<int>(ctx->n);
    const int npg = prec == 0 ? 256 : 512;      // as ising_solve_lowp pads
    const int np = (n + npg - 1) / npg * npg;
    const int Rp = (R + 63) / 64 * 64;
    char kb[256];
    std::snprintf(kb, sizeof(kb), "lowp-v2|%s|cus=%d|%s|np=%d|Rp=%d|iters=%lld", prop.gcnArchName,
                  prop.multiProcessorCount, prec == 0 ? "bf16" : "fp8", np, Rp, static_cast<long long>(iters));
    const std::string key(kb);
    auto report = [&](const doch::LowpShape& sh, double ms, int cached) {
        if (shape_out) {
            shape_out[0] = sh.bn;
            shape_out[1] = sh.splits;
            shape_out[2] = sh.sb;
            shape_out[3] = sh.depth;
        }
        if (ms_out) *ms_out = ms;
        if (from_cache_out) *from_cache_out = cached;
    };
    int v[4];
    double cms = 0.0;
    if (cache_lookup_ints(cache_path, key, kLowpFields, 4, v, &cms)) {
        doch::LowpShape sh;
        sh.bn = v[0];
        sh.splits = v[1];
        sh.sb = v[2];
        sh.depth = v[3];
        if (doch::lowp_shape_valid(prec, np, Rp, sh)) {
            ctx->lp_shape = sh;
            report(sh, cms, 1);
            return ISING_OK;
        }
    }
    // candidates: J held in LDS over its slice widths, the fused iteration,
    // and the split product over tile widths, splits, stage widths and
    // depths, as far as they fit
    std::vector<doch::LowpShape> cand;
    for (int sb : {1024, 512, 256}) {
        doch::LowpShape sh;
        sh.bn = 128;
        sh.splits = -2;
        sh.sb = sb;
        sh.depth = 1;
        if (doch::lowp_shape_valid(prec, np, Rp, sh)) cand.push_back(sh);
    }
    for (int mode : {-1, 0})
        for (int d : {2, 3}) {
            doch::LowpShape sh;
            sh.bn = 64;
            sh.splits = mode;
            sh.sb = 256;
            sh.depth = d;
            if (doch::lowp_shape_valid(prec, np, Rp, sh)) cand.push_back(sh);
        }
    for (int bn : {128, 64})
        for (int S : {1, 2, 4, 8})
            for (int sb : {128, 256})
                for (int d : {2, 3}) {
                    doch::LowpShape sh;
                    sh.bn = bn;
                    sh.splits = S;
                    sh.sb = sb;
                    sh.depth = d;
                    if (doch::lowp_shape_valid(prec, np, Rp, sh)) cand.push_back(sh);
                }
    if (cand.empty()) return fail(ISING_E_UNSUPPORTED, "no low-precision shape fits n=%d, R=%d", n, R);
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0), "event");
    HIP_OK(hipEventCreate(&e1), "event");
    const doch::LowpShape saved = ctx->lp_shape;
    doch::LowpShape best;
    double best_ms = -1.0;
    ising_status st = ISING_OK;
    for (const auto& sh : cand) {
        ctx->lp_shape = sh;
        // one run to allocate and warm up, one timed
        st = ising_solve_lowp(ctx, x0_dev, R, iters, params, jx_dtype, nullptr, nullptr, nullptr, nullptr, stream);
        if (st != ISING_OK) break;
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            st = ising_solve_lowp(ctx, x0_dev, R, iters, params, jx_dtype, nullptr, nullptr, nullptr, nullptr,
                                  stream);
            if (st != ISING_OK) break;
            e = hipEventRecord(e1, s);
        }
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune timing");
            break;
        }
        if (best_ms < 0.0 || ms < best_ms) {
            best_ms = ms;
            best = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ISING_OK) {
        ctx->lp_shape = saved;
        return st;
    }
    ctx->lp_shape = best;
    report(best, best_ms, 0);
    const int bv[4] = {best.bn, best.splits, best.sb, best.depth};
    (void)cache_store_ints(cache_path, key, kLowpFields, 4, bv, best_ms);
    return ISING_OK;
}

ising_status ising_set_lowp_shape(ising_ctx* ctx, int32_t bn, int32_t splits, int32_t stage_bytes,
                                  int32_t depth) {
    if (!ctx) return fail(ISING_E_INVALID_ARG, "NULL context");
    if (bn == 0) {
        ctx->lp_shape = doch::LowpShape{};
        return ISING_OK;
    }
    doch::LowpShape sh;
    sh.bn = bn;
    sh.splits = splits;
    sh.sb = stage_bytes;
    sh.depth = depth;
    // the values the library is built for; whether they fit a problem is
    // checked per call
    if (bn != 64 && bn != 128) return fail(ISING_E_INVALID_ARG, "bn must be 0, 64 or 128");
    if (splits != -2 && splits != -1 && splits != 0 && splits != 1 && splits != 2 && splits != 4 && splits != 8)
        return fail(ISING_E_INVALID_ARG, "splits must be -2, -1, 0, 1, 2, 4 or 8");
    if (splits == -2) {
        if (bn != 128 || depth != 1 || (stage_bytes != 256 && stage_bytes != 512 && stage_bytes != 1024))
            return fail(ISING_E_INVALID_ARG, "J held in LDS (splits -2) takes bn 128, depth 1 and slices of "
                                             "256, 512 or 1024 bytes");
        ctx->lp_shape = sh;
        return ISING_OK;
    }
    if (stage_bytes != 128 && stage_bytes != 256) return fail(ISING_E_INVALID_ARG, "stage_bytes must be 128 or 256");
    if (depth != 2 && depth != 3) return fail(ISING_E_INVALID_ARG, "depth must be 2 or 3");
    if (splits <= 0 && (bn != 64 || stage_bytes != 256))
        return fail(ISING_E_INVALID_ARG, "the fused iteration (splits 0 or -1) takes bn 64 and 256-byte stages");
    ctx->lp_shape = sh;
    return ISING_OK;
}

ising_status ising_set_batch_shape(ising_ctx* ctx, int32_t rj, int32_t wg, int32_t chunk_rows) {
    if (!ctx || !ctx->batch) return fail(ISING_E_INVALID_ARG, "not a batch context");
    if (rj == 0 && wg == 0 && chunk_rows == 0) {      // back to the default
        ctx->bshape_set = false;
        return ISING_OK;
    }
    doch::BatchShape sh;
    sh.rj = rj;
    sh.wg = wg;
    sh.chunk_rows = chunk_rows;
    if (!doch::batch_shape_supported(sh, rj))
        return fail(ISING_E_INVALID_ARG, "no batch kernel for %d restarts per unit on %d threads (chunks of %d rows)",
                    rj, wg, chunk_rows);
    ctx->bshape = sh;
    ctx->bshape_set = true;
    return ISING_OK;
}

}  // extern "C"

namespace {

// The tuning cache is a JSON object with one entry per line, the key then
// named integer fields and the time of the chosen shape,
//   "key": {"rj": 8, "wg": 256, "chunk_rows": 512, "ms": 12.5},
// written and read only by the functions below.
bool cache_lookup_ints(const char* path, const std::string& key, const char* const* names, int n, int* vals,
                       double* ms) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    const std::string head = "\"" + key + "\": {";
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        const char* p = std::strstr(line, head.c_str());
        if (!p) continue;
        p += head.size();
        bool ok = true;
        std::vector<int> v(static_cast<size_t>(n));
        for (int i = 0; i < n && ok; ++i) {
            const std::string field = "\"" + std::string(names[i]) + "\": ";
            const char* q = std::strstr(p, field.c_str());
            ok = q && std::sscanf(q + field.size(), "%d", &v[static_cast<size_t>(i)]) == 1;
        }
        const char* q = ok ? std::strstr(p, "\"ms\": ") : nullptr;
        double t = 0.0;
        if (q && std::sscanf(q + 6, "%lf", &t) == 1) {
            for (int i = 0; i < n; ++i) vals[i] = v[static_cast<size_t>(i)];
            *ms = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

bool cache_store_ints(const char* path, const std::string& key, const char* const* names, int n, const int* vals,
                      double ms) {
    if (!path) return false;
    std::vector<std::string> entries;
    const std::string head = "\"" + key + "\": {";
    if (FILE* f = std::fopen(path, "r")) {
        char line[1024];
        while (std::fgets(line, sizeof(line), f)) {
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == '\r' || l.back() == ',' || l.back() == ' '))
                l.pop_back();
            if (l.size() < 2 || l[0] != '"' || l.find(head) == 0) continue;
            entries.push_back(l);
        }
        std::fclose(f);
    }
    std::string e = head;
    char buf[96];
    for (int i = 0; i < n; ++i) {
        std::snprintf(buf, sizeof(buf), "\"%s\": %d, ", names[i], vals[i]);
        e += buf;
    }
    std::snprintf(buf, sizeof(buf), "\"ms\": %.4f}", ms);
    e += buf;
    entries.push_back(e);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fputs("{\n", f);
    for (size_t i = 0; i < entries.size(); ++i)
        std::fprintf(f, "%s%s\n", entries[i].c_str(), i + 1 < entries.size() ? "," : "");
    std::fputs("}\n", f);
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

const char* const kBatchFields[3] = {"rj", "wg", "chunk_rows"};
extern const char* const kLowpFields[4] = {"bn", "splits", "stage_bytes", "depth"};

bool cache_lookup(const char* path, const std::string& key, doch::BatchShape* sh, double* ms) {
    int v[3];
    if (!cache_lookup_ints(path, key, kBatchFields, 3, v, ms)) return false;
    sh->rj = v[0];
    sh->wg = v[1];
    sh->chunk_rows = v[2];
    return true;
}

bool cache_store(const char* path, const std::string& key, const doch::BatchShape& sh, double ms) {
    const int v[3] = {sh.rj, sh.wg, sh.chunk_rows};
    return cache_store_ints(path, key, kBatchFields, 3, v, ms);
}

}  // namespace

extern "C" {

ising_status ising_autotune_batch(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t max_iters,
                                  const double* alpha_host, const double* beta_host, double eps, int32_t x_dtype,
                                  const char* cache_path, void* stream, int32_t* shape_out, double* ms_out,
                                  int32_t* from_cache_out) {
    if (!ctx || !ctx->batch) return fail(ISING_E_INVALID_ARG, "not a batch context");
    if (!doch::batch_restarts_supported(R)) return fail(ISING_E_INVALID_ARG, "R must be 1, 2, 4, 8, 16 or 32");
    if (R > 8) return fail(ISING_E_UNSUPPORTED, "more than 8 restarts run one workgroup per instance: nothing to tune");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, ctx->device), "device properties");
    int64_t rows = 0, nnz = 0;
    for (const auto& I : ctx->inst_host) {
        rows += I.n;
        nnz += I.nnz;
    }
    char kb[512];
    std::snprintf(kb, sizeof(kb), "batch-v2|%s|cus=%d|count=%d|rows=%lld|nnz=%lld|R=%d|x=%s|v=%s|iters=%lld|eps=%.6g",
                  prop.gcnArchName, prop.multiProcessorCount, ctx->count, static_cast<long long>(rows),
                  static_cast<long long>(nnz), R, x_dtype == ISING_F64 ? "f64" : "f32",
                  ctx->vt == ISING_F64 ? "f64" : "f32", static_cast<long long>(max_iters), eps);
    const std::string key(kb);
    doch::BatchShape best;
    double best_ms = 0.0;
    if (cache_lookup(cache_path, key, &best, &best_ms) && doch::batch_shape_supported(best, R)) {
        ctx->bshape = best;
        ctx->bshape_set = true;
        if (shape_out) {
            shape_out[0] = best.rj;
            shape_out[1] = best.wg;
            shape_out[2] = best.chunk_rows;
        }
        if (ms_out) *ms_out = best_ms;
        if (from_cache_out) *from_cache_out = 1;
        return ISING_OK;
    }
    // candidates: restart groups and threads the kernel is built for,
    // chunks of 256 to 2048 rows
    std::vector<doch::BatchShape> cand;
    const int rjs[4] = {8, 4, 2, 1};
    const int wgs[3] = {256, 512, 1024};
    const int rpms[4] = {256, 512, 1024, 2048};
    for (int rj : rjs) {
        if (rj > R) continue;
        for (int wg : wgs)
            for (int rpm : rpms) {
                doch::BatchShape sh;
                sh.rj = rj;
                sh.wg = wg;
                sh.chunk_rows = rpm;
                if (doch::batch_shape_supported(sh, R)) cand.push_back(sh);
            }
    }
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0), "event");
    HIP_OK(hipEventCreate(&e1), "event");
    const doch::BatchShape saved = ctx->bshape;
    const bool saved_set = ctx->bshape_set;
    best_ms = -1.0;
    ising_status st = ISING_OK;
    for (const auto& sh : cand) {
        ctx->bshape = sh;
        ctx->bshape_set = true;
        // one run to capture and load, one timed
        st = ising_solve_batch(ctx, x0_dev, R, max_iters, alpha_host, beta_host, eps, x_dtype, nullptr, nullptr,
                               nullptr, nullptr, stream);
        if (st != ISING_OK) break;
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            st = ising_solve_batch(ctx, x0_dev, R, max_iters, alpha_host, beta_host, eps, x_dtype, nullptr, nullptr,
                                   nullptr, nullptr, stream);
            if (st != ISING_OK) break;
            e = hipEventRecord(e1, s);
        }
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune timing");
            break;
        }
        if (best_ms < 0.0 || ms < best_ms) {
            best_ms = ms;
            best = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ISING_OK || best_ms < 0.0) {
        ctx->bshape = saved;
        ctx->bshape_set = saved_set;
        return st != ISING_OK ? st : fail(ISING_E_UNSUPPORTED, "no batch shape to try");
    }
    ctx->bshape = best;
    ctx->bshape_set = true;
    if (shape_out) {
        shape_out[0] = best.rj;
        shape_out[1] = best.wg;
        shape_out[2] = best.chunk_rows;
    }
    if (ms_out) *ms_out = best_ms;
    if (from_cache_out) *from_cache_out = 0;
    (void)cache_store(cache_path, key, best, best_ms);
    return ISING_OK;
}

ising_status ising_solve_lowp(ising_ctx* ctx, const double* x0_dev, int32_t R, int64_t iters,
                              const ising_params* params, int32_t jx_dtype, double* x_out_dev,
                              int8_t* s_out_dev, double* H_final_dev, ising_stats* stats_host,
                              void* stream) {
    if (!ctx || !params || !x0_dev) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (!ctx->dense || ctx->proc_kind != 0)
        return fail(ISING_E_UNSUPPORTED, "the low-precision path needs a stored dense context");
    if (ctx->has_field) return fail(ISING_E_UNSUPPORTED, "the low-precision path takes no field");
    if (jx_dtype != ISING_BF16 && jx_dtype != ISING_FP8_E4M3)
        return fail(ISING_E_INVALID_ARG, "jx_dtype must be ISING_BF16 or ISING_FP8_E4M3");
    if (R < 1 || R > kMaxR) return fail(ISING_E_INVALID_ARG, "R=%d out of range", R);
    if (iters < 0) return fail(ISING_E_INVALID_ARG, "iters < 0");
    const ising_params& p = *params;
    if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return fail(ISING_E_INVALID_ARG, "alpha must be finite and > 0");
    if (!(p.beta > 0.0) || !std::isfinite(p.beta)) return fail(ISING_E_INVALID_ARG, "beta must be finite and > 0");
    if (!(p.eps >= 0.0)) return fail(ISING_E_INVALID_ARG, "eps must be >= 0");
    if (ctx->n > 65536) return fail(ISING_E_UNSUPPORTED, "the low-precision path is limited to n <= 65536");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int prec = jx_dtype == ISING_BF16 ? 0 : 1;
    const int n = static_cast<int>(ctx->n);
    // padded order: at least two whole 256-byte stages per row (512 k in FP8)
    const int npg = prec == 0 ? 256 : 512;
    const int np = (n + npg - 1) / npg * npg;
    const int Rp = (R + 63) / 64 * 64;
    const size_t esz = prec == 0 ? 2 : 1;
    if (!ctx->jq[prec]) {
        HIP_OK(dev_alloc(&ctx->jq[prec], static_cast<size_t>(np) * np * esz), "hipMalloc(Jq)");
        if (prec == 1) {
            HIP_OK(dev_alloc(&ctx->rscale, static_cast<size_t>(np) * sizeof(float)), "hipMalloc(scale)");
            HIP_OK(dev_alloc(&ctx->rowabs, static_cast<size_t>(np) * sizeof(double)), "hipMalloc(row sums)");
            HIP_OK(dev_alloc(&ctx->lp_cs, 3 * kMaxR * sizeof(float)), "hipMalloc(restart scales)");
            HIP_OK(dev_alloc(&ctx->lp_colmax, kMaxR * sizeof(unsigned int)), "hipMalloc(column maxima)");
        }
        HIP_OK(doch::launch_lowp_convert(prec, ctx->J, n, np, ctx->jq[prec], ctx->rscale, ctx->rowabs, s),
               "convert J");
        if (prec == 1) {
            // once per context: the bound that carries the restart scales
            std::vector<double> ra(static_cast<size_t>(np));
            HIP_OK(hipMemcpyAsync(ra.data(), ctx->rowabs, np * sizeof(double), hipMemcpyDeviceToHost, s),
                   "copy row sums");
            HIP_OK(hipStreamSynchronize(s), "sync");
            double m = 0.0;
            for (double v : ra) m = std::max(m, v);
            ctx->lp_rho_q = m;
        }
    }
    // three rotating iterate buffers (FP32 master and low-precision copy): a
    // restart that stops keeps its last iterate in buffer iters_done mod 3
    const size_t ubytes = static_cast<size_t>(np) * Rp * sizeof(float);
    const size_t ubbytes = static_cast<size_t>(np) * Rp * esz;
    if (!ctx->lp_u[0] || ctx->lp_ubytes < ubytes) {
        for (auto& b : ctx->lp_u) dev_free(b);
        ctx->lp_ubytes = 0;
        for (auto& b : ctx->lp_u) HIP_OK(dev_alloc(&b, ubytes), "hipMalloc(U)");
        ctx->lp_ubytes = ubytes;
    }
    if (!ctx->lp_ub[0] || ctx->lp_ubbytes < ubbytes) {
        for (auto& b : ctx->lp_ub) dev_free(b);
        ctx->lp_ubbytes = 0;
        for (auto& b : ctx->lp_ub) HIP_OK(dev_alloc(&b, ubbytes), "hipMalloc(Ub)");
        ctx->lp_ubbytes = ubbytes;
    }
    // two partial-sum buffers: iteration k writes one while its launch closes
    // iteration k - 1 from the other
    const size_t pstride = static_cast<size_t>(np / 64) * Rp * 4;
    HIP_OK(ensure(&ctx->lp_partials, &ctx->lp_pbytes, 2 * pstride * sizeof(double)), "hipMalloc(partials)");
    doch::LowpShape shape = ctx->lp_shape;
    if (shape.bn == 0 || !doch::lowp_shape_valid(prec, np, Rp, shape)) {
        int cus = 256;
        HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device), "CU count");
        shape = doch::lowp_default_shape(prec, np, Rp, cus);
    }
    HIP_OK(ensure(&ctx->lp_P, &ctx->lp_Pbytes, doch::lowp_product_bytes(prec, np, Rp, shape)), "hipMalloc(products)");
    if (!ctx->ticket) {
        HIP_OK(dev_alloc(&ctx->ticket, (kMaxR + 8 * doch::kSchedStride) * sizeof(unsigned int)), "hipMalloc(ticket)");
        HIP_OK(dev_alloc(&ctx->state, kMaxR * sizeof(RestartState)), "hipMalloc(state)");
        ctx->state_cap = kMaxR;
    }
    HIP_OK(ensure(&ctx->log, &ctx->log_bytes, static_cast<size_t>(std::max<int64_t>(iters, 1)) * R * 2 * sizeof(double)),
           "hipMalloc(log)");
    HIP_OK(doch::launch_init_state(ctx->state, R, ctx->ticket, nullptr, s), "init");
    const double sb = std::sqrt(p.beta);
    float* cs[3] = {ctx->lp_cs, ctx->lp_cs ? ctx->lp_cs + kMaxR : nullptr, ctx->lp_cs ? ctx->lp_cs + 2 * kMaxR : nullptr};
    HIP_OK(doch::launch_lowp_load(prec, x0_dev, n, R, np, Rp, sb, ctx->lp_colmax, cs[0], ctx->lp_u[0],
                                  ctx->lp_ub[0], s), "load");
    // the other buffers start as copies, so padding rows and restarts hold
    // finite values in every buffer
    for (int b = 1; b < 3; ++b) {
        HIP_OK(hipMemcpyAsync(ctx->lp_u[b], ctx->lp_u[0], ubytes, hipMemcpyDeviceToDevice, s), "copy U");
        HIP_OK(hipMemcpyAsync(ctx->lp_ub[b], ctx->lp_ub[0], ubbytes, hipMemcpyDeviceToDevice, s), "copy Ub");
        if (prec == 1)
            HIP_OK(hipMemcpyAsync(cs[b], cs[0], kMaxR * sizeof(float), hipMemcpyDeviceToDevice, s), "copy scales");
    }
    bool resident_done = false;
    auto fused_shape = [&]() {
        int cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
        return doch::lowp_default_shape(prec, np, Rp, cus);
    };
    // the resident runs count barrier arrivals (barriers x workgroups per
    // XCD) in 32-bit words: longer runs take the fused iteration as launches
    if (shape.splits == -1 && iters > 100000000) shape.splits = 0;
    if (shape.splits == -2) {
        const int64_t groups = static_cast<int64_t>(np / 128) * (static_cast<int64_t>(np) * esz / shape.sb);
        if (iters * 2 * ((groups + 7) / 8) >= (int64_t{1} << 31)) shape = fused_shape();
    }
    if (shape.splits == -2 && iters > 0) {
        // J held in LDS for the whole run, or the fused iteration a launch at
        // a time when the workgroups do not fit on the device at once
        if (!ctx->rsync) HIP_OK(dev_alloc(&ctx->rsync, sizeof(doch::ResidentSync)), "hipMalloc(sync)");
        HIP_OK(doch::launch_resident_reset(ctx->rsync, s), "reset");
        double* parts[2] = {ctx->lp_partials, ctx->lp_partials + pstride};
        void* ubs[3] = {ctx->lp_ub[0], ctx->lp_ub[1], ctx->lp_ub[2]};
        const hipError_t e = doch::launch_lowp_held(prec, np, Rp, shape, iters, ctx->jq[prec], ctx->rscale, ctx->lp_u,
                                                    ubs, cs, ctx->lp_rho_q, p.alpha, p.beta, p.eps, R, ctx->lp_P,
                                                    parts, ctx->log, ctx->state, ctx->rsync, s);
        if (e == hipSuccess) {
            resident_done = true;
        } else if (e == hipErrorCooperativeLaunchTooLarge) {
            (void)hipGetLastError();
            shape = fused_shape();
        } else {
            return hip_fail(e, "low-precision run with J held in LDS");
        }
    }
    if (shape.splits == -1 && iters > 0) {
        // the whole run in one cooperative launch, or the same iteration a
        // launch at a time when its grid does not fit on the device at once
        if (!ctx->rsync) HIP_OK(dev_alloc(&ctx->rsync, sizeof(doch::ResidentSync)), "hipMalloc(sync)");
        HIP_OK(doch::launch_resident_reset(ctx->rsync, s), "reset");
        double* parts[2] = {ctx->lp_partials, ctx->lp_partials + pstride};
        void* ubs[3] = {ctx->lp_ub[0], ctx->lp_ub[1], ctx->lp_ub[2]};
        const hipError_t e = doch::launch_lowp_resident(prec, np, Rp, shape, iters, ctx->jq[prec], ctx->rscale,
                                                        ctx->lp_u, ubs, cs, ctx->lp_rho_q, p.alpha, p.beta, p.eps, R,
                                                        parts, ctx->log, ctx->state, ctx->rsync, s);
        if (e == hipSuccess) {
            resident_done = true;
        } else if (e == hipErrorCooperativeLaunchTooLarge) {
            (void)hipGetLastError();
            shape.splits = 0;
        } else {
            return hip_fail(e, "resident low-precision run");
        }
    }
    for (int64_t k = 0; !resident_done && k < iters; ++k) {
        const int a = static_cast<int>(k % 3), b = static_cast<int>((k + 1) % 3);
        double* pk = ctx->lp_partials + (k & 1) * pstride;
        const double* pprev = ctx->lp_partials + ((k + 1) & 1) * pstride;
        HIP_OK(doch::launch_lowp_step(prec, np, Rp, shape, ctx->jq[prec], ctx->rscale, ctx->lp_u[a], ctx->lp_u[b],
                                      ctx->lp_ub[a], ctx->lp_ub[b], cs[a], cs[b], ctx->lp_rho_q, p.alpha, p.beta,
                                      p.eps, R, k, ctx->lp_P, pprev, pk, ctx->log, ctx->state, s),
               "low-precision step");
    }
    if (iters > 0)
        HIP_OK(doch::launch_lowp_close(np, Rp, R, iters - 1, ctx->lp_partials + ((iters - 1) & 1) * pstride,
                                       p.alpha, p.beta, p.eps, ctx->log, ctx->state, s),
               "close last iteration");
    ctx->last_R = R;
    ctx->last_iters = iters;
    double* xtmp = nullptr;
    if (x_out_dev || s_out_dev || H_final_dev) {
        double* xo = x_out_dev;
        if (!xo && H_final_dev) {
            HIP_OK(dev_alloc(&xtmp, static_cast<size_t>(n) * R * sizeof(double)), "hipMalloc(x)");
            xo = xtmp;
        }
        hipError_t e = doch::launch_lowp_finish(ctx->lp_u, ctx->state, n, R, Rp, sb, xo, s_out_dev, s);
        if (e == hipSuccess && H_final_dev) {
            // per (row tile of 64, padded restart) three FP64 partial sums
            Scratch sc;
            ising_status st = ensure_scratch(ctx, static_cast<size_t>((n + 63) / 64) * Rp * 3, &sc);
            if (st != ISING_OK) { dev_free(xtmp); return st; }
            e = doch::launch_dense_objective(ctx->J, n, R, xo, p.alpha, p.beta, sc.partials, sc.tickets,
                                             H_final_dev, s);
        }
        if (e != hipSuccess) { dev_free(xtmp); return hip_fail(e, "finish"); }
    }
    if (xtmp) {
        (void)hipStreamSynchronize(s);
        dev_free(xtmp);
    }
    // a timed-out barrier wait of the resident run is reported here
    return read_stats(ctx, R, stats_host, s);
}

ising_status ising_get_log(ising_ctx* ctx, int32_t restart, int64_t first, int64_t count,
                           double* H_host, double* r_host, void* stream) {
    if (!ctx) return fail(ISING_E_INVALID_ARG, "ctx is NULL");
    if (restart < 0 || restart >= std::max(ctx->last_R, 1)) return fail(ISING_E_INVALID_ARG, "bad restart");
    if (first < 0 || count < 0 || first + count > ctx->last_iters)
        return fail(ISING_E_INVALID_ARG, "log range outside the last solve");
    if (count == 0) return ISING_OK;
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int R = ctx->last_R;
    std::vector<double> buf(static_cast<size_t>(count) * R * 2);
    HIP_OK(hipMemcpyAsync(buf.data(), ctx->log + static_cast<size_t>(first) * R * 2,
                          buf.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy log");
    HIP_OK(hipStreamSynchronize(s), "sync");
    for (int64_t k = 0; k < count; ++k) {
        if (H_host) H_host[k] = buf[(static_cast<size_t>(k) * R + restart) * 2];
        if (r_host) r_host[k] = buf[(static_cast<size_t>(k) * R + restart) * 2 + 1];
    }
    return ISING_OK;
}

}  // extern "C"

namespace {

// Argument checks of ising_energy and the size of its launch: the grid and
// the partial sums the kernel that launch_*_energy picks needs.
ising_status energy_plan(const ising_ctx* ctx, const int8_t* s_dev, int32_t R, const double* E_dev,
                         const int64_t* E_int_dev, int* grid_out, size_t* need_out) {
    if (!ctx) return fail(ISING_E_INVALID_ARG, "ctx is NULL");
    if (!s_dev) return fail(ISING_E_INVALID_ARG, "s is NULL");
    if (R < 1 || R > kMaxR) return fail(ISING_E_INVALID_ARG, "R=%d out of range", R);
    if (!E_dev && !E_int_dev) return fail(ISING_E_INVALID_ARG, "no output requested");
    if (E_int_dev && !ctx->integer_J) return fail(ISING_E_UNSUPPORTED, "integer energy needs integer couplings");
    if (E_int_dev && ctx->dense) return fail(ISING_E_UNSUPPORTED, "integer energy is computed for CSR contexts only");
    if (ctx->dense && !E_dev) return fail(ISING_E_INVALID_ARG, "E is NULL");
    const int grid = ctx->dense ? std::min<int64_t>(1024, (ctx->n + 3) / 4)
                                : std::min<int64_t>(1024, (ctx->n + 255) / 256);
    size_t need;
    if (!ctx->dense) {
        // per (workgroup, restart): J part, field part, integer J part
        need = (R >= 2 && R <= 8) ? static_cast<size_t>(doch::csr_energy8_grid(ctx->n)) * R * 3
                                  : static_cast<size_t>(grid) * R * 3;
    } else if (ctx->proc_kind == 1 && !ctx->h) {
        // generated couplings: per (restart rounded up to its block of 8, workgroup)
        need = static_cast<size_t>(grid) * ((R + 7) / 8 * 8);
    } else if (R >= doch::kTiledEnergyMinR) {
        // per (64-row tile, restart padded to 64): J part, field part
        need = static_cast<size_t>((ctx->n + 63) / 64) * ((R + 63) / 64 * 64) * 2;
    } else {
        need = static_cast<size_t>(grid) * R * 2;
    }
    *grid_out = grid;
    *need_out = need;
    return ISING_OK;
}

ising_status energy_launch(const ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* E_dev,
                           int64_t* E_int_dev, double* partials, unsigned int* tickets, int grid,
                           hipStream_t s) {
    if (ctx->dense)
        HIP_OK(doch::launch_dense_energy(dense_view(ctx), s_dev, R, partials, tickets, grid, E_dev, s), "energy");
    else
        HIP_OK(doch::launch_csr_energy(csr_view(ctx), s_dev, R, partials, tickets, grid, E_dev, E_int_dev, s),
               "energy");
    return ISING_OK;
}

// ---------------------------------------------------- allocation-free energy
// The partial sums and tickets of ising_energy_noalloc live in this array,
// one copy per device, held until the process ends.  Host code never uses
// the array's name as an address: the device address of each device's copy
// is looked up once, with that device current, and kept in g_scratch_addr.
constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr size_t kScratchTicketBytes = kMaxR * sizeof(unsigned int);
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kScratchMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
ising_status scratch_address(int device, unsigned char** out) {
    if (device < 0 || device >= kScratchMaxDevices)
        return fail(ISING_E_UNSUPPORTED, "device %d beyond the %d the library tracks", device, kScratchMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(ISING_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_addr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_addr[device]);
    return ISING_OK;
}

// Zero the tickets: every energy kernel counts arrivals from 0.  A kernel
// rather than a memset node keeps the call safe to capture in a graph.
__global__ void zero_tickets_kernel(unsigned int* t, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) t[i] = 0u;
}

}  // namespace

extern "C" {

ising_status ising_energy(ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* E_dev,
                          int64_t* E_int_dev, void* stream) {
    int grid = 0;
    size_t need = 0;
    ising_status st = energy_plan(ctx, s_dev, R, E_dev, E_int_dev, &grid, &need);
    if (st != ISING_OK) return st;
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    Scratch sc;
    st = ensure_scratch(ctx, need, &sc);
    if (st != ISING_OK) return st;
    return energy_launch(ctx, s_dev, R, E_dev, E_int_dev, sc.partials, sc.tickets, grid,
                         static_cast<hipStream_t>(stream));
}

ising_status ising_energy_noalloc(ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* E_dev,
                                  int64_t* E_int_dev, void* stream) {
    int grid = 0;
    size_t need = 0;
    ising_status st = energy_plan(ctx, s_dev, R, E_dev, E_int_dev, &grid, &need);
    if (st != ISING_OK) return st;
    if (ctx->batch) return fail(ISING_E_UNSUPPORTED, "use ising_energy_batch on a batch context");
    const size_t cap = (kScratchBytes - kScratchTicketBytes) / sizeof(double);
    if (need > cap)
        return fail(ISING_E_INVALID_ARG,
                    "n=%lld with R=%d needs %zu partial sums; the static scratch of ising_energy_noalloc "
                    "holds %zu (%zu bytes)",
                    static_cast<long long>(ctx->n), R, need, cap, kScratchBytes);
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    unsigned char* base = nullptr;
    st = scratch_address(ctx->device, &base);
    if (st != ISING_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned int* tickets = reinterpret_cast<unsigned int*>(base);
    double* partials = reinterpret_cast<double*>(base + kScratchTicketBytes);
    hipLaunchKernelGGL(zero_tickets_kernel, dim3(4), dim3(256), 0, s, tickets, kMaxR);
    HIP_OK(hipGetLastError(), "zero tickets");
    return energy_launch(ctx, s_dev, R, E_dev, E_int_dev, partials, tickets, grid, s);
}


ising_status ising_cut(ising_ctx* ctx, const int8_t* s_dev, int32_t R, double* cut_dev, int64_t* cut_int_dev,
                       void* stream) {
    if (!ctx) return fail(ISING_E_INVALID_ARG, "ctx is NULL");
    if (!s_dev) return fail(ISING_E_INVALID_ARG, "s is NULL");
    if (R < 1 || R > kMaxR) return fail(ISING_E_INVALID_ARG, "R=%d out of range", R);
    if (!cut_dev && !cut_int_dev) return fail(ISING_E_INVALID_ARG, "no output requested");
    if (ctx->has_field) return fail(ISING_E_UNSUPPORTED, "the cut is defined for h = 0");
    if (ctx->batch) return fail(ISING_E_UNSUPPORTED, "cuts of batch contexts are not provided");
    if (cut_int_dev && (!ctx->integer_J || ctx->dense))
        return fail(ISING_E_UNSUPPORTED, "the exact cut needs integer CSR couplings");
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ctx->cut_tmp) HIP_OK(dev_alloc(&ctx->cut_tmp, 2 * kMaxR * sizeof(double)), "hipMalloc(cut)");
    double* E = ctx->cut_tmp;
    int64_t* Ei = reinterpret_cast<int64_t*>(ctx->cut_tmp + kMaxR);
    ising_status st = ising_energy(ctx, s_dev, R, E, cut_int_dev ? Ei : nullptr, stream);
    if (st != ISING_OK) return st;
    // S_J: pass 0 of the statistics kernels (sum of the stored off-diagonal couplings)
    const int grid = 1024;
    Scratch sc;
    st = ensure_scratch(ctx, static_cast<size_t>(2048) * 4, &sc);
    if (st != ISING_OK) return st;
    if (ctx->dense)
        HIP_OK(doch::launch_dense_stats(dense_view(ctx), 0.0, 0, sc.partials, sc.tickets, grid, sc.stats, s), "stats");
    else
        HIP_OK(doch::launch_csr_stats(csr_view(ctx), 0.0, 0, sc.partials, sc.tickets, grid, sc.stats, s), "stats");
    HIP_OK(doch::launch_cut(E, cut_int_dev ? Ei : nullptr, sc.stats, R, cut_dev, cut_int_dev, s), "cut");
    HIP_OK(hipStreamSynchronize(s), "sync");
    return ISING_OK;
}


ising_status ising_tune_eta(ising_ctx* ctx, const double* x0_dev, int32_t count, const double* etas_host,
                            int64_t probe_iters, int32_t method, void* stream, ising_params* best_out,
                            double* best_eta_out, double* energies_host) {
    if (!ctx || !x0_dev || !etas_host || !best_out) return fail(ISING_E_INVALID_ARG, "NULL argument");
    if (ctx->batch) return fail(ISING_E_UNSUPPORTED, "use ising_default_params_batch on a batch context");
    if (count < 1 || count > 64) return fail(ISING_E_INVALID_ARG, "count must be 1..64");
    if (probe_iters < 1 || probe_iters > 1000) return fail(ISING_E_INVALID_ARG, "probe_iters must be 1..1000");
    for (int k = 0; k < count; ++k)
        if (!(etas_host[k] > 0.0) || !(etas_host[k] <= 2.0))
            return fail(ISING_E_INVALID_ARG, "eta[%d] must be in (0, 2]", k);
    HIP_OK(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // lambda_hat and the row-sum bound once (eq:alphabeta), then each eta
    ising_params p1;
    ising_status st = ising_default_params(ctx, 1.0, method, stream, &p1, nullptr);
    if (st != ISING_OK) return st;
    const double lambda = ctx->last_lambda, rowsum = ctx->last_rowsum;
    const double np = static_cast<double>(ctx->np);
    if (!ctx->cut_tmp) HIP_OK(dev_alloc(&ctx->cut_tmp, 2 * kMaxR * sizeof(double)), "hipMalloc(energies)");
    std::vector<ising_params> ps(static_cast<size_t>(count), p1);
    std::vector<double> Es(static_cast<size_t>(count), 0.0);
    for (int k = 0; k < count; ++k) {
        ps[k].alpha = etas_host[k] * lambda;
        ps[k].beta = std::pow(np, 1.5) * (ps[k].alpha + rowsum);
    }
    // CSR, and procedural dense couplings: up to 8 probes at a time as
    // restarts of one pass over the couplings (each probe's iterates are
    // those ising_solve computes)
    const bool proc_sweep = ctx->dense && ctx->proc_kind == 1 && !ctx->has_field;
    if (!ctx->dense || proc_sweep) {
        const int rmax = std::min<int>(count, doch::kSweepMaxR);
        HIP_OK(ensure(&ctx->sweep_x, &ctx->sweep_x_bytes, 2 * static_cast<size_t>(ctx->np) * rmax * sizeof(double)),
               "hipMalloc(sweep iterates)");
        HIP_OK(ensure(&ctx->tune_s, &ctx->tune_s_bytes, static_cast<size_t>(ctx->n) * rmax), "hipMalloc(spins)");
        const int grid = proc_sweep ? doch::dense_sweep_grid(ctx->n) : doch::sweep_grid(ctx->n);
        HIP_OK(ensure(&ctx->partials, &ctx->partials_bytes,
                      static_cast<size_t>(grid) * rmax * doch::kNumPartials * sizeof(double)),
               "hipMalloc(partials)");
        st = ensure_solve_state(ctx, 1, rmax);
        if (st != ISING_OK) return st;
        const CsrView cv = proc_sweep ? CsrView{} : csr_view(ctx);
        for (int c0 = 0; c0 < count; c0 += doch::kSweepMaxR) {
            const int R = std::min(doch::kSweepMaxR, count - c0);
            if (R == 1) {
                // a lone probe runs on the single-restart path
                st = ising_solve(ctx, x0_dev, 1, probe_iters, &ps[c0], nullptr, ctx->tune_s, nullptr, stream);
                if (st != ISING_OK) return st;
                st = ising_energy(ctx, ctx->tune_s, 1, ctx->cut_tmp, nullptr, stream);
                if (st != ISING_OK) return st;
                HIP_OK(hipMemcpyAsync(Es.data() + c0, ctx->cut_tmp, sizeof(double), hipMemcpyDeviceToHost, s),
                       "copy energy");
                continue;
            }
            double* X[2] = {ctx->sweep_x, ctx->sweep_x + static_cast<size_t>(ctx->np) * R};
            HIP_OK(doch::launch_init_state(ctx->state, R, ctx->ticket, nullptr, s), "init");
            HIP_OK(doch::launch_sweep_load(x0_dev, ctx->np, R, X[0], s), "load sweep");
            doch::SweepArgs a{};
            a.R = R;
            for (int r = 0; r < R; ++r) {
                a.alpha[r] = ps[c0 + r].alpha;
                a.beta[r] = ps[c0 + r].beta;
            }
            a.partials = ctx->partials;
            a.tickets = ctx->ticket;
            a.state = ctx->state;
            for (int64_t k = 0; k < probe_iters; ++k) {
                a.x_old = X[k & 1];
                a.x_new = X[(k + 1) & 1];
                a.k = k;
                if (proc_sweep) HIP_OK(doch::launch_dense_sin_sweep(ctx->n, ctx->proc_seed, a, s), "sweep step");
                else HIP_OK(doch::launch_sweep_step(cv, a, s), "sweep step");
            }
            HIP_OK(doch::launch_sweep_round(X[probe_iters & 1], ctx->n, R, ctx->has_field, ctx->tune_s, s), "round");
            st = ising_energy(ctx, ctx->tune_s, R, ctx->cut_tmp, nullptr, stream);
            if (st != ISING_OK) return st;
            HIP_OK(hipMemcpyAsync(Es.data() + c0, ctx->cut_tmp, R * sizeof(double), hipMemcpyDeviceToHost, s),
                   "copy energies");
        }
        HIP_OK(hipStreamSynchronize(s), "sync");
    } else {
        HIP_OK(ensure(&ctx->tune_s, &ctx->tune_s_bytes, static_cast<size_t>(ctx->n)), "hipMalloc(spins)");
        for (int k = 0; k < count; ++k) {
            st = ising_solve(ctx, x0_dev, 1, probe_iters, &ps[k], nullptr, ctx->tune_s, nullptr, stream);
            if (st != ISING_OK) return st;
            st = ising_energy(ctx, ctx->tune_s, 1, ctx->cut_tmp, nullptr, stream);
            if (st != ISING_OK) return st;
            HIP_OK(hipMemcpyAsync(Es.data() + k, ctx->cut_tmp, sizeof(double), hipMemcpyDeviceToHost, s),
                   "copy energy");
        }
        HIP_OK(hipStreamSynchronize(s), "sync");
    }
    int best = 0;
    for (int k = 0; k < count; ++k) {
        if (energies_host) energies_host[k] = Es[k];
        if (Es[k] < Es[best]) best = k;
    }
    const ising_params best_p = ps[best];
    *best_out = best_p;
    if (best_eta_out) *best_eta_out = etas_host[best];
    return ISING_OK;
}

}  // extern "C"
