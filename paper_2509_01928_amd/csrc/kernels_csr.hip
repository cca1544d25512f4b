// kernels_csr.hip -- sparse (CSR) kernels of the DOCH hot path for gfx950.
//
// One DOCH iteration (Methods, eq:FPE / Alg. 1) on a CSR coupling matrix is a
// single streaming pass: row blocks of up to 512 rows and 2045 stored
// entries are assigned to workgroups; a workgroup streams the block's column
// indices and values as 16-byte non-temporal chunks (they are used once per
// iteration, so they should not evict the iterate from L2), all requested
// before the first is used, gathers the iterate, parks the products in LDS,
// and then one thread per row sums its products in ascending column order,
// applies the cube-root update and adds to the iteration's FP64 partial
// sums.  The last workgroup finishes the iteration (H, r, the field spin) --
// see step_common.h.
//
// Blocks are dealt out XCD-aware: workgroup w runs on XCD w mod 8, and XCD c
// owns the contiguous c-th eighth of the blocks, so the rows being gathered
// by one XCD's workgroups at any moment are neighbours and their iterate
// entries are reused in that XCD's private L2.
#include "device_common.h"
#include "ising_internal.h"
#include "step_common.h"

namespace doch {

namespace {

constexpr int NT = kBlockThreads;
constexpr int NW = NT / kWave;

__device__ __forceinline__ void block_range(int64_t nblk, int64_t& b, int64_t& bend,
                                            int64_t& bstep) {
    const unsigned G = gridDim.x;
    if ((G & 7u) == 0 && nblk >= static_cast<int64_t>(G)) {
        const unsigned xcd = blockIdx.x & 7u;
        const unsigned slot = blockIdx.x >> 3;
        b = nblk * xcd / 8 + slot;
        bend = nblk * (xcd + 1) / 8;
        bstep = G >> 3;
    } else {
        b = blockIdx.x;
        bend = nblk;
        bstep = G;
    }
}

// Registers of one row block in flight: its bounds and every value the
// block's rows need from HBM, requested by issue_block() one block ahead of
// its use.
template <typename XT, typename VT, typename HT, int CH, int RPT>
struct Stage {
    int r0, r1, e0, e1;
    typename Vec4<int>::type cv[CH];
    typename Vec4<VT>::type vv[CH];
    int rpv[RPT];
    XT xi[RPT];
    HT hv[RPT];
};

template <int CH, int RPT>
struct Geometry {
    static constexpr int rows = NT * RPT;
    static constexpr int span = 4 * NT * CH;
};

template <typename XT, typename VT, typename HT, bool FIELD, int CH, int RPT>
__device__ __forceinline__ void issue_block(Stage<XT, VT, HT, CH, RPT>& s, int64_t b,
                                            const int2* __restrict__ binfo,
                                            const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ col,
                                            const VT* __restrict__ val,
                                            const HT* __restrict__ h, const XT* __restrict__ x) {
    const int2 m0 = binfo[b], m1 = binfo[b + 1];
    s.r0 = m0.x;
    s.e0 = m0.y;
    s.r1 = m1.x;
    s.e1 = m1.y;
    const int ea = s.e0 & ~3;
    if (s.e1 - ea > Geometry<CH, RPT>::span) return;      // long row: loaded on its own
    const int t = static_cast<int>(threadIdx.x);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int base = ea + 4 * (t + NT * u);
        if (base < s.e1) {
            s.cv[u] = ld_stream4(col + base);
            s.vv[u] = ld_stream4(val + base);
        }
    }
    const int nr = s.r1 - s.r0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int rr = t + q * NT;
        if (rr < nr) {
            s.rpv[q] = ld_stream(rp + s.r0 + rr);
            s.xi[q] = x[s.r0 + rr];
            if (FIELD) s.hv[q] = ld_stream(h + s.r0 + rr);
        }
    }
}

// Process the block held in `cur`; the loads of the next block (if any) are
// issued into `nxt` after the current gathers, so they overlap this block's
// gathers, LDS traffic and arithmetic without delaying them.
template <typename XT, typename VT, typename HT, bool FIELD, int CH, int RPT>
__device__ __forceinline__ void process_block(
    Stage<XT, VT, HT, CH, RPT>& cur, Stage<XT, VT, HT, CH, RPT>& nxt, bool has_next,
    int64_t nb, const int2* __restrict__ binfo, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const VT* __restrict__ val, const HT* __restrict__ h,
    const XT* __restrict__ x, XT* __restrict__ xn, double t_old, const StepArgs& a,
    double* prod, int* rps, double* red, double (&acc)[kNumPartials]) {
    using G = Geometry<CH, RPT>;
    const int t = static_cast<int>(threadIdx.x);
    const int cnt = cur.e1 - cur.e0;
    const int ea = cur.e0 & ~3;
    if (cur.e1 - ea <= G::span) {
        XT g[CH][4];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int base = ea + 4 * (t + NT * u);
            if (base < cur.e1) {
                g[u][0] = x[cur.cv[u].x];
                g[u][1] = x[cur.cv[u].y];
                g[u][2] = x[cur.cv[u].z];
                g[u][3] = x[cur.cv[u].w];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (has_next) issue_block<XT, VT, HT, FIELD, CH, RPT>(nxt, nb, binfo, rp, col, val, h, x);
        __builtin_amdgcn_sched_barrier(0);
        const int nr = cur.r1 - cur.r0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int rr = t + q * NT;
            if (rr < nr) rps[rr] = cur.rpv[q];
        }
        if (t == 0) rps[nr] = cur.e1;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int base = ea + 4 * (t + NT * u);
            if (base < cur.e1) {
                double* p = prod + (base - ea);
                p[0] = dmul(static_cast<double>(cur.vv[u].x), static_cast<double>(g[u][0]));
                p[1] = dmul(static_cast<double>(cur.vv[u].y), static_cast<double>(g[u][1]));
                p[2] = dmul(static_cast<double>(cur.vv[u].z), static_cast<double>(g[u][2]));
                p[3] = dmul(static_cast<double>(cur.vv[u].w), static_cast<double>(g[u][3]));
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int rr = t + q * NT;
            if (rr < nr) {
                const int lo = rps[rr] - ea, hi = rps[rr + 1] - ea;
                double z = 0.0;
                for (int e = lo; e < hi; ++e) z = dadd(z, prod[e]);
                const double hq = FIELD ? static_cast<double>(cur.hv[q]) : 0.0;
                if (FIELD) z = dadd(z, dmul(hq, t_old));
                update_row<XT>(z, static_cast<double>(cur.xi[q]), hq, FIELD, a, xn, cur.r0 + rr, acc);
            }
        }
        __syncthreads();
    } else {
        if (has_next) issue_block<XT, VT, HT, FIELD, CH, RPT>(nxt, nb, binfo, rp, col, val, h, x);
        // one long row: the whole workgroup reduces it
        const int r0 = cur.r0, e0 = cur.e0;
        double part[1] = {0.0};
        for (int e = t; e < cnt; e += NT) {
            const int c = ld_stream(col + e0 + e);
            const double v = static_cast<double>(ld_stream(val + e0 + e));
            part[0] = dadd(part[0], dmul(v, static_cast<double>(x[c])));
        }
        block_sum<1, NT>(part, red);
        if (t == 0) {
            double z = part[0];
            double hr = 0.0;
            if (FIELD) {
                hr = static_cast<double>(h[r0]);
                z = dadd(z, dmul(hr, t_old));
            }
            update_row<XT>(z, static_cast<double>(x[r0]), hr, FIELD, a, xn, r0, acc);
        }
        __syncthreads();
    }
}

// DYN = false: workgroup w takes every (G/8)-th block of its XCD's range.
// DYN = true: the workgroups of an XCD take the blocks of its range in order
// from a shared counter, each claiming the block after next while it works,
// so an XCD's workgroups stay on neighbouring blocks (their gathered iterate
// entries stay in that XCD's L2) and finish together.
template <typename XT, typename VT, typename HT, bool FIELD, int CH, int RPT, bool DYN>
__global__ __launch_bounds__(NT) void csr_step_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h,
    const int2* __restrict__ binfo, int64_t nblk, StepArgs a) {
    if (a.state->done) return;
    using G = Geometry<CH, RPT>;
    __shared__ double prod[G::span];
    __shared__ int rps[G::rows + 1];
    __shared__ double red[kNumPartials * NW];
    __shared__ int64_t queue[2];
    const XT* __restrict__ x = static_cast<const XT*>(a.x_old);
    XT* __restrict__ xn = static_cast<XT*>(a.x_new);
    const double t_old = FIELD ? static_cast<double>(x[n]) : 0.0;
    double acc[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;

    int64_t b, bend, bstep, nb;
    block_range(nblk, b, bend, bstep);
    unsigned int* counter = nullptr;
    int64_t start = 0;
    if (DYN) {
        const bool chunked = (gridDim.x & 7u) == 0 && nblk >= static_cast<int64_t>(gridDim.x);
        const unsigned xcd = chunked ? (blockIdx.x & 7u) : 0u;
        start = chunked ? nblk * xcd / 8 : 0;
        counter = a.sched + xcd * kSchedStride;
        if (threadIdx.x == 0) {
            queue[0] = start + atomicAdd(counter, 1u);
            queue[1] = start + atomicAdd(counter, 1u);
        }
        __syncthreads();
        b = queue[0];
        nb = queue[1];
        __syncthreads();
    } else {
        nb = b + bstep;
    }
    Stage<XT, VT, HT, CH, RPT> sa, sb;
    if (b < bend) issue_block<XT, VT, HT, FIELD, CH, RPT>(sa, b, binfo, rp, col, val, h, x);
    // two stages alternate roles, so no register copy waits on a load; with
    // DYN each half publishes its claim through its own LDS slot, read after
    // process_block's closing barrier
    while (b < bend) {
        if (DYN && threadIdx.x == 0) queue[0] = nb < bend ? start + atomicAdd(counter, 1u) : bend;
        process_block<XT, VT, HT, FIELD, CH, RPT>(sa, sb, nb < bend, nb, binfo, rp, col, val, h, x,
                                                  xn, t_old, a, prod, rps, red, acc);
        b = nb;
        nb = DYN ? queue[0] : b + bstep;
        if (b >= bend) break;
        if (DYN && threadIdx.x == 0) queue[1] = nb < bend ? start + atomicAdd(counter, 1u) : bend;
        process_block<XT, VT, HT, FIELD, CH, RPT>(sb, sa, nb < bend, nb, binfo, rp, col, val, h, x,
                                                  xn, t_old, a, prod, rps, red, acc);
        b = nb;
        nb = DYN ? queue[1] : b + bstep;
    }
    step_epilogue<XT, NT>(a, acc, red, n, FIELD, t_old);
}

// Lane-per-row variant for short rows.  Each lane owns U rows at a time
// (rows i, i + S, ..., S = threads in the grid) and loads a row's entries as
// up to MAXC aligned 16-byte chunks straight into registers -- no LDS, no
// barriers, no block table.  Rows that need more chunks fall back to an
// element loop.  Sums still run in ascending column order.  The whole grid
// sweeps the rows together, so at any moment every stream is read within one
// narrow window of addresses: measured on MI355X this streams the lattice
// faster than giving each XCD its own eighth of the rows, and a row's
// neighbours one lattice row away are still inside the window when it is
// gathered.
// RL: 0 = row offsets read from rp; -1 = every row holds row_len entries
// (row i starts at row_len i, rp not read); d > 0 = the same with row_len = d
// known at compile time (d = 4: the 4-neighbour lattice).
// CT: int32_t = column indices; int16_t = each entry's cyclic column offset
// (col - i taken into [-32768, 32767] modulo n), decoded back to the column.
template <typename XT, typename VT, typename HT, bool FIELD, int U, int MAXC, int RL, typename CT = int32_t>
__global__ __launch_bounds__(NT) void csr_rowlane_kernel(
    int64_t n, const int32_t* __restrict__ rp, const CT* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, int row_len, StepArgs a) {
    if (a.state->done) return;
    __shared__ double red[kNumPartials * NW];
    const XT* __restrict__ x = static_cast<const XT*>(a.x_old);
    XT* __restrict__ xn = static_cast<XT*>(a.x_new);
    const double t_old = FIELD ? static_cast<double>(x[n]) : 0.0;
    double acc[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;

    const int64_t hi = n;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * NT;
    // column of row i's entry whose stored index is c
    auto column = [n](int64_t i, int c) -> int64_t {
        if constexpr (sizeof(CT) == 4) {
            return c;
        } else {
            int64_t j = i + c;
            j += j < 0 ? n : 0;
            j -= j >= n ? n : 0;
            return j;
        }
    };
    for (int64_t base = first; base < hi; base += stride * U) {
        int s[U], e[U], a0[U];
        XT xi[U];
        HT hv[U];
        typename Vec4<CT>::type cv[U][MAXC];
        typename Vec4<VT>::type vv[U][MAXC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * stride;
            if (i < hi) {
                if (RL != 0) {                  // constant row length: offsets implicit
                    const int d = RL > 0 ? RL : row_len;
                    s[u] = static_cast<int>(i * d);
                    e[u] = s[u] + d;
                } else {
                    s[u] = rp[i];
                    e[u] = rp[i + 1];
                }
                xi[u] = x[i];
                if (FIELD) hv[u] = ld_stream(h + i);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * stride;
            if (i < hi) {
                a0[u] = s[u] & ~3;
#pragma unroll
                for (int c = 0; c < MAXC; ++c) {
                    if (a0[u] + 4 * c < e[u]) {
                        cv[u][c] = ld_stream4(col + a0[u] + 4 * c);
                        vv[u][c] = ld_stream4(val + a0[u] + 4 * c);
                    }
                }
            }
        }
        XT g[U][MAXC][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * stride;
            if (i < hi) {
#pragma unroll
                for (int c = 0; c < MAXC; ++c) {
                    const int b0 = a0[u] + 4 * c;
                    if (b0 < e[u]) {
                        const int cc[4] = {cv[u][c].x, cv[u][c].y, cv[u][c].z, cv[u][c].w};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (b0 + q >= s[u] && b0 + q < e[u]) g[u][c][q] = x[column(i, cc[q])];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * stride;
            if (i < hi) {
                double z = 0.0;
                if (e[u] - a0[u] <= 4 * MAXC) {
#pragma unroll
                    for (int c = 0; c < MAXC; ++c) {
                        const int b0 = a0[u] + 4 * c;
                        const double vd[4] = {static_cast<double>(vv[u][c].x), static_cast<double>(vv[u][c].y),
                                              static_cast<double>(vv[u][c].z), static_cast<double>(vv[u][c].w)};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (b0 + q >= s[u] && b0 + q < e[u])
                                z = dadd(z, dmul(vd[q], static_cast<double>(g[u][c][q])));
                    }
                } else {
                    for (int k = s[u]; k < e[u]; ++k)
                        z = dadd(z, dmul(static_cast<double>(val[k]), static_cast<double>(x[column(i, col[k])])));
                }
                const double hq = FIELD ? static_cast<double>(hv[u]) : 0.0;
                if (FIELD) z = dadd(z, dmul(hq, t_old));
                update_row<XT>(z, static_cast<double>(xi[u]), hq, FIELD, a, xn, i, acc);
            }
        }
    }
    step_epilogue<XT, NT>(a, acc, red, n, FIELD, t_old);
}

// ---------------------------------------------------------------- energy
// eq:IsingModel for restart blockIdx.y: E = -1/2 sum_i s_i (J s)_i - h.s
template <typename VT, typename HT, bool FIELD>
__global__ __launch_bounds__(NT) void csr_energy_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, const int8_t* __restrict__ s,
    int R, int want_int, double* partials, unsigned int* tickets, double* E,
    int64_t* E_int) {
    __shared__ double red[3 * NW];
    __shared__ int64_t redi[NW];
    __shared__ int last_flag;
    const int r = blockIdx.y;
    double eJ = 0.0, eh = 0.0;
    int64_t eI = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        double acc = 0.0;
        int64_t iacc = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const double sj = static_cast<double>(s[static_cast<int64_t>(col[e]) * R + r]);
            const double v = static_cast<double>(val[e]);
            acc = dadd(acc, dmul(v, sj));
            if (want_int) iacc += static_cast<int64_t>(v) * static_cast<int64_t>(sj);
        }
        const double si = static_cast<double>(s[i * R + r]);
        eJ = dadd(eJ, dmul(si, acc));
        eI += static_cast<int64_t>(si) * iacc;
        if (FIELD) eh = dadd(eh, dmul(static_cast<double>(h[i]), si));
    }
    double v[2] = {eJ, eh};
    block_sum<2, NT>(v, red);
    int64_t wi = wave_sum_i64(eI);
    if ((threadIdx.x & (kWave - 1)) == 0) redi[threadIdx.x / kWave] = wi;
    __syncthreads();
    double* p = partials + (static_cast<size_t>(r) * gridDim.x + blockIdx.x) * 3;
    if (threadIdx.x == 0) {
        int64_t ti = 0;
        for (int w = 0; w < NW; ++w) ti += redi[w];
        store_agent(p + 0, v[0]);
        store_agent(p + 1, v[1]);
        store_agent(p + 2, __longlong_as_double(ti));
        last_flag = arrive_last(tickets + r, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[2] = {0.0, 0.0};
    int64_t ui = 0;
    const double* pr = partials + static_cast<size_t>(r) * gridDim.x * 3;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT) {
        u[0] = dadd(u[0], load_agent(pr + g * 3 + 0));
        u[1] = dadd(u[1], load_agent(pr + g * 3 + 1));
        ui += __double_as_longlong(load_agent(pr + g * 3 + 2));
    }
    block_sum<2, NT>(u, red);
    int64_t wu = wave_sum_i64(ui);
    if ((threadIdx.x & (kWave - 1)) == 0) redi[threadIdx.x / kWave] = wu;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t ti = 0;
        for (int w = 0; w < NW; ++w) ti += redi[w];
        if (E) E[r] = dsub(dmul(-0.5, u[0]), u[1]);
        if (E_int) E_int[r] = -(ti / 2);
        reset_ticket(tickets + r);
    }
}

// The same for 2 <= R <= 8 restarts in one pass over the couplings: eight
// lanes per row, lane r holding restart r, so the spins of a column are one
// run of R bytes and the row's entries are read once for all restarts.  The
// last workgroup adds the workgroups' sums of each restart in index order.
template <typename VT, typename HT, bool FIELD, int R>
__global__ __launch_bounds__(NT) void csr_energy8_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, const int8_t* __restrict__ s,
    int want_int, double* partials, unsigned int* tickets, double* E, int64_t* E_int) {
    constexpr int G = 8;
    __shared__ double redd[NW][G][2];
    __shared__ int64_t redi[NW][G];
    __shared__ int last_flag;
    const int r = threadIdx.x & (G - 1);
    const bool on = r < R;
    double eJ = 0.0, eh = 0.0;
    int64_t eI = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * (NT / G) + threadIdx.x / G; i < n;
         i += static_cast<int64_t>(gridDim.x) * (NT / G)) {
        double acc = 0.0;
        int64_t iacc = 0;
        const int e1 = rp[i + 1];
        for (int e = rp[i]; e < e1; ++e) {
            const double v = static_cast<double>(val[e]);
            const double sj = on ? static_cast<double>(s[static_cast<int64_t>(col[e]) * R + r]) : 0.0;
            acc = dadd(acc, dmul(v, sj));
            if (want_int) iacc += static_cast<int64_t>(v) * static_cast<int64_t>(sj);
        }
        if (!on) continue;
        const double si = static_cast<double>(s[i * R + r]);
        eJ = dadd(eJ, dmul(si, acc));
        eI += static_cast<int64_t>(si) * iacc;
        if (FIELD) eh = dadd(eh, dmul(static_cast<double>(h[i]), si));
    }
    // per restart: the wavefront's eight row groups, then the wavefronts in order
#pragma unroll
    for (int off = 8; off < kWave; off <<= 1) {
        eJ = dadd(eJ, __shfl_xor(eJ, off, kWave));
        eh = dadd(eh, __shfl_xor(eh, off, kWave));
        eI += __shfl_xor(eI, off, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane < G) {
        redd[wave][lane][0] = eJ;
        redd[wave][lane][1] = eh;
        redi[wave][lane] = eI;
    }
    __syncthreads();
    if (threadIdx.x < R) {
        double tJ = 0.0, th = 0.0;
        int64_t ti = 0;
        for (int w = 0; w < NW; ++w) {
            tJ = dadd(tJ, redd[w][threadIdx.x][0]);
            th = dadd(th, redd[w][threadIdx.x][1]);
            ti += redi[w][threadIdx.x];
        }
        double* p = partials + (static_cast<size_t>(blockIdx.x) * R + threadIdx.x) * 3;
        store_agent(p + 0, tJ);
        store_agent(p + 1, th);
        store_agent(p + 2, __longlong_as_double(ti));
    }
    // the storing wavefront (0) waits for its stores inside the arrival
    if (threadIdx.x == 0) last_flag = arrive_last_grid(tickets, gridDim.x) ? 1 : 0;
    __syncthreads();
    if (!last_flag) return;
    if (threadIdx.x < R) {
        double uJ = 0.0, uh = 0.0;
        int64_t ui = 0;
        for (unsigned g = 0; g < gridDim.x; ++g) {
            const double* p = partials + (static_cast<size_t>(g) * R + threadIdx.x) * 3;
            uJ = dadd(uJ, load_agent(p + 0));
            uh = dadd(uh, load_agent(p + 1));
            ui += __double_as_longlong(load_agent(p + 2));
        }
        if (E) E[threadIdx.x] = dsub(dmul(-0.5, uJ), uh);
        if (E_int) E_int[threadIdx.x] = -(ui / 2);
    }
    if (threadIdx.x == 0) reset_ticket(tickets);
}

// ------------------------------------------------------------ validation
// flags[0]: malformed CSR, flags[1]: nonzero diagonal, flags[2]: a value is
// not an integer of magnitude < 2^31, flags[3]: a value is not an integer in
// [-128, 127], flags[4]: an entry's cyclic column offset (col - i modulo n,
// taken into [-32768, 32767]) does not fit 16 bits.
template <typename VT>
__global__ __launch_bounds__(NT) void csr_validate_kernel(
    int64_t n, int64_t nnz, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, int32_t* flags) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        const int64_t a = rp[i], b = rp[i + 1];
        if ((i == 0 && a != 0) || b < a || (i == n - 1 && b != nnz) || b > nnz || a < 0) {
            atomicOr(flags + 0, 1);
            continue;
        }
        int prev = -1;
        for (int64_t e = a; e < b; ++e) {
            const int c = col[e];
            if (c < 0 || c >= n || c <= prev) atomicOr(flags + 0, 1);
            prev = c;
            const double v = static_cast<double>(val[e]);
            if (c == i && v != 0.0) atomicOr(flags + 1, 1);
            if (!(v == floor(v)) || fabs(v) >= 2147483648.0) atomicOr(flags + 2, 1);
            if (!(v == floor(v)) || v < -128.0 || v > 127.0) atomicOr(flags + 3, 1);
            int64_t d = static_cast<int64_t>(c) - i;
            if (d > 32767) d -= n;
            else if (d < -32768) d += n;
            if (d > 32767 || d < -32768) atomicOr(flags + 4, 1);
        }
    }
}

// every stored (i, j, v) needs a stored (j, i, v)
template <typename VT>
__global__ __launch_bounds__(NT) void csr_symcheck_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, int32_t* bad) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = col[e];
            int lo = rp[j], hi = rp[j + 1] - 1;
            bool found = false;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = col[mid];
                if (c == i) {
                    found = (val[mid] == val[e]);
                    break;
                }
                if (c < i) lo = mid + 1; else hi = mid - 1;
            }
            if (!found) atomicOr(bad, 1);
        }
    }
}

// --------------------------------------------------------- matrix stats
// pass 0: max_i sum_{j!=i}|Jhat_ij|, sum Jhat_ij, #stored, sum |h|
// pass 1: sum over stored off-diagonal entries of (Jhat_ij - mean)^2
template <typename VT, typename HT, bool FIELD>
__global__ __launch_bounds__(NT) void csr_stats_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, double mean, int pass,
    double* partials, unsigned int* ticket, MatrixStats* out) {
    __shared__ double red[3 * NW];
    __shared__ double redm[NW];
    __shared__ int last_flag;
    double pmax = 0.0, s1 = 0.0, cnt = 0.0, habs = 0.0, ss = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        double rs = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] == i) continue;
            const double v = static_cast<double>(val[e]);
            if (pass == 0) {
                rs = dadd(rs, fabs(v));
                s1 = dadd(s1, v);
                cnt += 1.0;
            } else {
                const double d = dsub(v, mean);
                ss = dadd(ss, dmul(d, d));
            }
        }
        if (FIELD) {
            const double hv = static_cast<double>(h[i]);
            if (pass == 0) {
                rs = dadd(rs, fabs(hv));
                s1 = dadd(s1, dmul(2.0, hv));
                cnt += 2.0;
                habs = dadd(habs, fabs(hv));
            } else {
                const double d = dsub(hv, mean);
                ss = dadd(ss, dmul(2.0, dmul(d, d)));
            }
        }
        pmax = fmax(pmax, rs);
    }
    double v[3];
    if (pass == 0) { v[0] = s1; v[1] = cnt; v[2] = habs; }
    else { v[0] = ss; v[1] = 0.0; v[2] = 0.0; }
    block_sum<3, NT>(v, red);
    double wm = wave_max(pmax);
    if ((threadIdx.x & (kWave - 1)) == 0) redm[threadIdx.x / kWave] = wm;
    __syncthreads();
    double* p = partials + static_cast<size_t>(blockIdx.x) * 4;
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < NW; ++w) m = fmax(m, redm[w]);
        store_agent(p + 0, v[0]);
        store_agent(p + 1, v[1]);
        store_agent(p + 2, v[2]);
        store_agent(p + 3, m);
        last_flag = arrive_last_grid(ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[3] = {0.0, 0.0, 0.0};
    double um = 0.0;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT) {
        u[0] = dadd(u[0], load_agent(partials + g * 4 + 0));
        u[1] = dadd(u[1], load_agent(partials + g * 4 + 1));
        u[2] = dadd(u[2], load_agent(partials + g * 4 + 2));
        um = fmax(um, load_agent(partials + g * 4 + 3));
    }
    block_sum<3, NT>(u, red);
    double wum = wave_max(um);
    if ((threadIdx.x & (kWave - 1)) == 0) redm[threadIdx.x / kWave] = wum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < NW; ++w) m = fmax(m, redm[w]);
        if (pass == 0) {
            const double rmax = FIELD ? fmax(m, u[2]) : m;   // row n sums |h_i|
            out->rowsum_max = rmax;
            out->abs_max = rmax;
            out->s1 = u[0];
            out->stored = u[1];
        } else {
            out->ss = u[0];
        }
        reset_ticket(ticket);
    }
}

// ---------------------------------------------------- power iteration step
// w = (c I - Jhat) v, with mu_log[2k] = v.w and mu_log[2k+1] = |w|_2.
template <typename VT, typename HT, bool FIELD>
__global__ __launch_bounds__(NT) void csr_power_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, double c,
    const double* __restrict__ v, double* __restrict__ w, double* partials,
    unsigned int* ticket, double* mu_log, int64_t k) {
    __shared__ double red[3 * NW];
    __shared__ int last_flag;
    const double vn = FIELD ? v[n] : 0.0;
    double acc[3] = {0.0, 0.0, 0.0};   // v.w, w.w, h.v
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        double z = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            z = dadd(z, dmul(static_cast<double>(val[e]), v[col[e]]));
        if (FIELD) {
            const double hv = static_cast<double>(h[i]);
            z = dadd(z, dmul(hv, vn));
            acc[2] = dadd(acc[2], dmul(hv, v[i]));
        }
        const double wi = dsub(dmul(c, v[i]), z);
        w[i] = wi;
        acc[0] = dadd(acc[0], dmul(v[i], wi));
        acc[1] = dadd(acc[1], dmul(wi, wi));
    }
    block_sum<3, NT>(acc, red);
    if (threadIdx.x == 0) {
        double* p = partials + static_cast<size_t>(blockIdx.x) * 3;
        for (int q = 0; q < 3; ++q) store_agent(p + q, acc[q]);
        last_flag = arrive_last_grid(ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[3] = {0.0, 0.0, 0.0};
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT)
        for (int q = 0; q < 3; ++q) u[q] = dadd(u[q], load_agent(partials + g * 3 + q));
    block_sum<3, NT>(u, red);
    if (threadIdx.x == 0) {
        double vw = u[0], ww = u[1];
        if (FIELD) {
            const double wn = dsub(dmul(c, vn), u[2]);
            w[n] = wn;
            vw = dadd(vw, dmul(vn, wn));
            ww = dadd(ww, dmul(wn, wn));
        }
        mu_log[2 * k] = vw;
        mu_log[2 * k + 1] = sqrt(ww);
        reset_ticket(ticket);
    }
}

int grid_for_rows(int64_t n) {
    int64_t g = (n + NT - 1) / NT;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

#define DOCH_DISPATCH_VT_HT(A, ...)                                               \
    do {                                                                          \
        if ((A).vt == ISING_I16 && (A).ht == ISING_F64) {                         \
            using VT = int16_t; using HT = double; __VA_ARGS__;                   \
        } else if ((A).vt == ISING_I16) {                                         \
            using VT = int16_t; using HT = float; __VA_ARGS__;                    \
        } else if ((A).vt == ISING_F64 && (A).ht == ISING_F64) {                  \
            using VT = double; using HT = double; __VA_ARGS__;                    \
        } else if ((A).vt == ISING_F64) {                                         \
            using VT = double; using HT = float; __VA_ARGS__;                     \
        } else if ((A).ht == ISING_F64) {                                         \
            using VT = float; using HT = double; __VA_ARGS__;                     \
        } else {                                                                  \
            using VT = float; using HT = float; __VA_ARGS__;                      \
        }                                                                         \
    } while (0)

namespace {

template <typename XT, typename VT, typename HT, bool FIELD, int CH, int RPT, bool DYN>
hipError_t launch_step_t(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    auto kern = csr_step_kernel<XT, VT, HT, FIELD, CH, RPT, DYN>;
    static int per_cu = 0;      // resident workgroups per CU for this instantiation
    static int cus = 0;
    if (per_cu == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        int occ = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, 0);
        if (e != hipSuccess) return e;
        per_cu = occ < 1 ? 1 : occ;
    }
    const int wpc = (plan.wg_per_cu > 0 && plan.wg_per_cu < per_cu) ? plan.wg_per_cu : per_cu;
    int64_t grid = static_cast<int64_t>(wpc) * cus;
    if (grid > kMaxStepGrid) grid = kMaxStepGrid;
    if (grid >= 8) grid &= ~static_cast<int64_t>(7);
    if (grid > plan.nblk) grid = plan.nblk;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(NT), 0, s, A.n, A.rp, A.col,
                       static_cast<const VT*>(A.val), static_cast<const HT*>(A.h), plan.binfo,
                       plan.nblk, a);
    return hipGetLastError();
}

template <typename XT, typename VT, typename HT, bool FIELD, int U, int MAXC, int RL, typename CT = int32_t>
hipError_t launch_rowlane_r(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    auto kern = csr_rowlane_kernel<XT, VT, HT, FIELD, U, MAXC, RL, CT>;
    const CT* colp;
    if constexpr (sizeof(CT) == 2) colp = A.col16;
    else colp = A.col;
    static int per_cu = 0;
    static int cus = 0;
    if (per_cu == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        int occ = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, 0);
        if (e != hipSuccess) return e;
        per_cu = occ < 1 ? 1 : occ;
    }
    const int wpc = (plan.wg_per_cu > 0 && plan.wg_per_cu < per_cu) ? plan.wg_per_cu : per_cu;
    int64_t grid = static_cast<int64_t>(wpc) * cus;
    if (grid > kMaxStepGrid) grid = kMaxStepGrid;
    const int64_t need = (A.n + NT - 1) / NT;           // one row per thread at most
    if (grid > need) grid = need;
    if (grid >= 8) grid &= ~static_cast<int64_t>(7);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(NT), 0, s, A.n, A.rp, colp,
                       static_cast<const VT*>(A.val), static_cast<const HT*>(A.h), A.row_len, a);
    return hipGetLastError();
}

template <typename XT, typename VT, typename HT, bool FIELD, int U, int MAXC>
hipError_t launch_rowlane_t(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    if (A.row_len == 4) return launch_rowlane_r<XT, VT, HT, FIELD, U, MAXC, 4>(A, plan, a, s);
    if (A.row_len > 0) return launch_rowlane_r<XT, VT, HT, FIELD, U, MAXC, -1>(A, plan, a, s);
    return launch_rowlane_r<XT, VT, HT, FIELD, U, MAXC, 0>(A, plan, a, s);
}

template <typename XT, typename VT, typename HT, bool FIELD>
hipError_t launch_step_geo(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    switch (plan.geometry) {
        case 0: return launch_step_t<XT, VT, HT, FIELD, 1, 1, false>(A, plan, a, s);
        case 1: return launch_step_t<XT, VT, HT, FIELD, 2, 2, false>(A, plan, a, s);
        case 2: return launch_step_t<XT, VT, HT, FIELD, 4, 2, false>(A, plan, a, s);
        case 3: return launch_rowlane_t<XT, VT, HT, FIELD, 1, 1>(A, plan, a, s);
        case 4: return launch_rowlane_t<XT, VT, HT, FIELD, 1, 2>(A, plan, a, s);
        case 5: return launch_step_t<XT, VT, HT, FIELD, 1, 1, true>(A, plan, a, s);
        case 6: return launch_step_t<XT, VT, HT, FIELD, 2, 2, true>(A, plan, a, s);
        default: return launch_step_t<XT, VT, HT, FIELD, 4, 2, true>(A, plan, a, s);
    }
}

template <typename XT, typename HT, bool FIELD>
hipError_t launch_rowlane_i8_f(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    CsrView B = A;
    B.val = A.val8;
    // 4-entry rows whose cyclic column offsets fit 16 bits: indices streamed
    // as those offsets too
    if (A.col16 && A.row_len == 4) {
        if (plan.geometry == 3) return launch_rowlane_r<XT, int8_t, HT, FIELD, 1, 1, 4, int16_t>(B, plan, a, s);
        return launch_rowlane_r<XT, int8_t, HT, FIELD, 1, 2, 4, int16_t>(B, plan, a, s);
    }
    if (plan.geometry == 3) return launch_rowlane_t<XT, int8_t, HT, FIELD, 1, 1>(B, plan, a, s);
    return launch_rowlane_t<XT, int8_t, HT, FIELD, 1, 2>(B, plan, a, s);
}

template <typename XT, typename HT>
hipError_t launch_rowlane_i8(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    if (A.h) return launch_rowlane_i8_f<XT, HT, true>(A, plan, a, s);
    return launch_rowlane_i8_f<XT, HT, false>(A, plan, a, s);
}

template <typename XT, typename VT, typename HT>
hipError_t launch_step_field(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    if (A.h) return launch_step_geo<XT, VT, HT, true>(A, plan, a, s);
    return launch_step_geo<XT, VT, HT, false>(A, plan, a, s);
}

}  // namespace

void csr_geometry(int geometry, int* rows, int* span) {
    switch (geometry) {
        case 0: case 5: *rows = Geometry<1, 1>::rows; *span = Geometry<1, 1>::span; break;
        case 1: case 6: *rows = Geometry<2, 2>::rows; *span = Geometry<2, 2>::span; break;
        case 2: case 7: *rows = Geometry<4, 2>::rows; *span = Geometry<4, 2>::span; break;
        default: *rows = 0; *span = 0; break;      // lane-per-row kernels use no blocks
    }
}

hipError_t launch_csr_step(const CsrView& A, const CsrPlan& plan, const StepArgs& a, hipStream_t s) {
    // small-integer couplings: the lane-per-row kernels stream the 8-bit copy
    // (a quarter of the FP32 value bytes; the products are the same, since
    // each value converts exactly)
    if (A.val8 && (plan.geometry == 3 || plan.geometry == 4)) {
        const bool f64x = a.x_dtype == ISING_F64;
        if (A.ht == ISING_F64)
            return f64x ? launch_rowlane_i8<double, double>(A, plan, a, s) : launch_rowlane_i8<float, double>(A, plan, a, s);
        return f64x ? launch_rowlane_i8<double, float>(A, plan, a, s) : launch_rowlane_i8<float, float>(A, plan, a, s);
    }
    DOCH_DISPATCH_VT_HT(A, {
        if (a.x_dtype == ISING_F64) return launch_step_field<double, VT, HT>(A, plan, a, s);
        return launch_step_field<float, VT, HT>(A, plan, a, s);
    });
    return hipErrorInvalidValue;
}

template <typename VT, typename HT, bool FIELD>
hipError_t launch_energy8_f(const CsrView& A, const int8_t* s_spins, int R, int want_int, double* partials,
                            unsigned int* ticket, double* E, int64_t* E_int, hipStream_t s) {
    const int g8 = csr_energy8_grid(A.n);
    const VT* val = static_cast<const VT*>(A.val);
    const HT* h = static_cast<const HT*>(A.h);
    switch (R) {
#define DOCH_ENERGY8(RR)                                                                                  \
    case RR:                                                                                              \
        hipLaunchKernelGGL((csr_energy8_kernel<VT, HT, FIELD, RR>), dim3(g8), dim3(NT), 0, s, A.n, A.rp,   \
                           A.col, val, h, s_spins, want_int, partials, ticket, E, E_int);                  \
        break;
        DOCH_ENERGY8(2)
        DOCH_ENERGY8(3)
        DOCH_ENERGY8(4)
        DOCH_ENERGY8(5)
        DOCH_ENERGY8(6)
        DOCH_ENERGY8(7)
        DOCH_ENERGY8(8)
#undef DOCH_ENERGY8
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename VT, typename HT>
hipError_t launch_energy8(const CsrView& A, const int8_t* s_spins, int R, bool field, int want_int,
                          double* partials, unsigned int* ticket, double* E, int64_t* E_int, hipStream_t s) {
    if (field) return launch_energy8_f<VT, HT, true>(A, s_spins, R, want_int, partials, ticket, E, E_int, s);
    return launch_energy8_f<VT, HT, false>(A, s_spins, R, want_int, partials, ticket, E, E_int, s);
}

int csr_energy8_grid(int64_t n) {
    int64_t g = (n + NT / 8 - 1) / (NT / 8);
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

hipError_t launch_csr_energy(const CsrView& A, const int8_t* s_spins, int R,
                             double* partials, unsigned int* ticket, int grid,
                             double* E, int64_t* E_int, hipStream_t s) {
    const bool field = A.h != nullptr;
    const int want_int = E_int != nullptr;
    if (R >= 2 && R <= 8) {
        DOCH_DISPATCH_VT_HT(A, {
            return launch_energy8<VT, HT>(A, s_spins, R, field, want_int, partials, ticket, E, E_int, s);
        });
        return hipGetLastError();
    }
    DOCH_DISPATCH_VT_HT(A, {
        const VT* val = static_cast<const VT*>(A.val);
        const HT* h = static_cast<const HT*>(A.h);
        if (field)
            hipLaunchKernelGGL((csr_energy_kernel<VT, HT, true>), dim3(grid, R), dim3(NT), 0, s,
                               A.n, A.rp, A.col, val, h, s_spins, R, want_int, partials, ticket, E, E_int);
        else
            hipLaunchKernelGGL((csr_energy_kernel<VT, HT, false>), dim3(grid, R), dim3(NT), 0, s,
                               A.n, A.rp, A.col, val, h, s_spins, R, want_int, partials, ticket, E, E_int);
    });
    return hipGetLastError();
}

hipError_t launch_csr_validate(const CsrView& A, int32_t* flags, hipStream_t s) {
    const int grid = grid_for_rows(A.n);
    if (A.vt == ISING_F64)
        hipLaunchKernelGGL(csr_validate_kernel<double>, dim3(grid), dim3(NT), 0, s, A.n, A.nnz,
                           A.rp, A.col, static_cast<const double*>(A.val), flags);
    else if (A.vt == ISING_I16)
        hipLaunchKernelGGL(csr_validate_kernel<int16_t>, dim3(grid), dim3(NT), 0, s, A.n, A.nnz,
                           A.rp, A.col, static_cast<const int16_t*>(A.val), flags);
    else
        hipLaunchKernelGGL(csr_validate_kernel<float>, dim3(grid), dim3(NT), 0, s, A.n, A.nnz,
                           A.rp, A.col, static_cast<const float*>(A.val), flags);
    return hipGetLastError();
}

namespace {
// out[e] = val[e] for values already checked to be integers in [-128, 127],
// so the conversion is exact.
template <typename VT>
__global__ __launch_bounds__(NT) void csr_pack_i8_kernel(int64_t nnz, const VT* __restrict__ val,
                                                         int8_t* __restrict__ out) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; e < nnz;
         e += static_cast<int64_t>(gridDim.x) * NT)
        out[e] = static_cast<int8_t>(static_cast<int>(val[e]));
}
}  // namespace

namespace {
// out[e] = row i's cyclic column offset of entry e (checked to fit 16 bits)
__global__ __launch_bounds__(NT) void csr_pack_col16_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            int16_t* __restrict__ out) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t d = static_cast<int64_t>(col[e]) - i;
            if (d > 32767) d -= n;
            else if (d < -32768) d += n;
            out[e] = static_cast<int16_t>(d);
        }
    }
}
}  // namespace

hipError_t launch_csr_pack_col16(const CsrView& A, int16_t* out, hipStream_t s) {
    hipLaunchKernelGGL(csr_pack_col16_kernel, dim3(grid_for_rows(A.n)), dim3(NT), 0, s, A.n, A.rp, A.col, out);
    return hipGetLastError();
}

hipError_t launch_csr_pack_i8(const CsrView& A, int8_t* out, hipStream_t s) {
    if (A.nnz <= 0) return hipSuccess;
    const int grid = grid_for_rows(A.nnz);
    if (A.vt == ISING_F64)
        hipLaunchKernelGGL(csr_pack_i8_kernel<double>, dim3(grid), dim3(NT), 0, s, A.nnz,
                           static_cast<const double*>(A.val), out);
    else if (A.vt == ISING_I16)
        hipLaunchKernelGGL(csr_pack_i8_kernel<int16_t>, dim3(grid), dim3(NT), 0, s, A.nnz,
                           static_cast<const int16_t*>(A.val), out);
    else
        hipLaunchKernelGGL(csr_pack_i8_kernel<float>, dim3(grid), dim3(NT), 0, s, A.nnz,
                           static_cast<const float*>(A.val), out);
    return hipGetLastError();
}

hipError_t launch_csr_symcheck(const CsrView& A, int32_t* bad, hipStream_t s) {
    const int grid = grid_for_rows(A.n);
    if (A.vt == ISING_F64)
        hipLaunchKernelGGL(csr_symcheck_kernel<double>, dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, static_cast<const double*>(A.val), bad);
    else if (A.vt == ISING_I16)
        hipLaunchKernelGGL(csr_symcheck_kernel<int16_t>, dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, static_cast<const int16_t*>(A.val), bad);
    else
        hipLaunchKernelGGL(csr_symcheck_kernel<float>, dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, static_cast<const float*>(A.val), bad);
    return hipGetLastError();
}

hipError_t launch_csr_stats(const CsrView& A, double mean, int pass, double* partials,
                            unsigned int* ticket, int grid, MatrixStats* out,
                            hipStream_t s) {
    const bool field = A.h != nullptr;
    DOCH_DISPATCH_VT_HT(A, {
        const VT* val = static_cast<const VT*>(A.val);
        const HT* h = static_cast<const HT*>(A.h);
        if (field)
            hipLaunchKernelGGL((csr_stats_kernel<VT, HT, true>), dim3(grid), dim3(NT), 0, s,
                               A.n, A.rp, A.col, val, h, mean, pass, partials, ticket, out);
        else
            hipLaunchKernelGGL((csr_stats_kernel<VT, HT, false>), dim3(grid), dim3(NT), 0, s,
                               A.n, A.rp, A.col, val, h, mean, pass, partials, ticket, out);
    });
    return hipGetLastError();
}

hipError_t launch_csr_power_step(const CsrView& A, double c, const double* v, double* w,
                                 double* partials, unsigned int* ticket, int grid,
                                 double* mu_log, int64_t k, hipStream_t s) {
    const bool field = A.h != nullptr;
    DOCH_DISPATCH_VT_HT(A, {
        const VT* val = static_cast<const VT*>(A.val);
        const HT* h = static_cast<const HT*>(A.h);
        if (field)
            hipLaunchKernelGGL((csr_power_kernel<VT, HT, true>), dim3(grid), dim3(NT), 0, s,
                               A.n, A.rp, A.col, val, h, c, v, w, partials, ticket, mu_log, k);
        else
            hipLaunchKernelGGL((csr_power_kernel<VT, HT, false>), dim3(grid), dim3(NT), 0, s,
                               A.n, A.rp, A.col, val, h, c, v, w, partials, ticket, mu_log, k);
    });
    return hipGetLastError();
}

}  // namespace doch
