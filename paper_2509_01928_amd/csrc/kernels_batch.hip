// kernels_batch.hip -- many independent instances x many restarts in one
// persistent launch.
//
// The instances are the diagonal blocks of one CSR matrix.  A workgroup pulls
// a whole instance from a work queue (instances ordered by decreasing size,
// so the long ones start first and the short ones fill the gaps) and runs
// the complete DOCH loop (eq:FPE / Alg. 1) on it for all R restarts at once:
// thread (slot, r) owns restart r of rows slot, slot + S, ... (S = threads /
// R), so the R iterate entries a coupling multiplies are contiguous
// (restart-interleaved storage) and J x for the R restarts is one pass over
// the instance's couplings -- a sparse matrix times an n x R block.  Every
// synchronisation is a workgroup barrier: instances never wait for each
// other.  Each restart stops on its own when r^(k) < eps (Remark S2): its
// iterate is frozen (copied forward) while the others go on; the instance
// ends when all its restarts have stopped or after max_iters iterations,
// and stamps the device clock for its time to solution.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "ising_internal.h"

namespace doch {

namespace {

constexpr int BT = kBatchThreads;
constexpr int BW = BT / kWave;

__device__ __forceinline__ uint64_t device_clock() { return __builtin_amdgcn_s_memrealtime(); }

// Sum v over the threads of the workgroup that share tid % R (R divides 64);
// thread r < R receives the total for restart r.  Fixed order.
template <int R, int K>
__device__ __forceinline__ void restart_sum(double (&v)[K], double* lds /* K*BW*R */) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < K; ++q) {
#pragma unroll
        for (int off = kWave / 2; off >= R; off >>= 1) v[q] = dadd(v[q], __shfl_xor(v[q], off, kWave));
    }
    if (lane < R) {
#pragma unroll
        for (int q = 0; q < K; ++q) lds[(q * BW + wave) * R + lane] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < R) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int w = 0; w < BW; ++w) s = dadd(s, lds[(q * BW + w) * R + threadIdx.x]);
            v[q] = s;
        }
    }
    __syncthreads();
}

template <typename XT, typename VT, int R>
__global__ __launch_bounds__(BT) void batch_solve_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const VT* __restrict__ val,
    const BatchInstance* __restrict__ inst, const int32_t* __restrict__ order, int count,
    const double* __restrict__ alpha, const double* __restrict__ beta, double eps,
    int64_t max_iters, const double* __restrict__ x0, XT* __restrict__ xa, XT* __restrict__ xb,
    unsigned int* queue, BatchRestartStat* __restrict__ stats, uint64_t* __restrict__ clock_start,
    uint64_t* __restrict__ clock_end, double* __restrict__ x_out, int8_t* __restrict__ s_out) {
    constexpr int S = BT / R;                 // row slots
    __shared__ double red[4 * BW * R];
    __shared__ int conv[R];
    __shared__ int s_job;
    __shared__ int s_all;
    const int r = threadIdx.x % R;
    const int slot = threadIdx.x / R;
    if (threadIdx.x == 0) atomicMin(reinterpret_cast<unsigned long long*>(clock_start),
                                    static_cast<unsigned long long>(device_clock()));
    for (;;) {
        if (threadIdx.x == 0) s_job = static_cast<int>(atomicAdd(queue, 1u));
        if (threadIdx.x < R) conv[threadIdx.x] = 0;
        __syncthreads();
        const int job = s_job;
        if (job >= count) break;
        const int k = order[job];
        const BatchInstance I = inst[k];
        const double a = alpha[k], b = beta[k];
        const int64_t base = static_cast<int64_t>(I.row0) * R;
        // start vectors into buffer a
        for (int64_t t = threadIdx.x; t < static_cast<int64_t>(I.n) * R; t += BT)
            xa[base + t] = static_cast<XT>(x0[base + t]);
        __syncthreads();
        const XT* xo = xa;
        XT* xw = xb;
        int64_t it = 0;
        int nonfinite = 0;
        for (; it < max_iters; ++it) {
            const bool frozen = conv[r] != 0;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};   // x^4, x^2, x z, (dx)^2
            for (int i = I.row0 + slot; i < I.row0 + I.n; i += S) {
                const int s = rp[i], e = rp[i + 1];
                double z = 0.0;
                int q = s;
                for (; q + 4 <= e; q += 4) {
                    const int c0 = col[q], c1 = col[q + 1], c2 = col[q + 2], c3 = col[q + 3];
                    const double v0 = static_cast<double>(val[q]), v1 = static_cast<double>(val[q + 1]);
                    const double v2 = static_cast<double>(val[q + 2]), v3 = static_cast<double>(val[q + 3]);
                    const double g0 = static_cast<double>(xo[static_cast<int64_t>(c0) * R + r]);
                    const double g1 = static_cast<double>(xo[static_cast<int64_t>(c1) * R + r]);
                    const double g2 = static_cast<double>(xo[static_cast<int64_t>(c2) * R + r]);
                    const double g3 = static_cast<double>(xo[static_cast<int64_t>(c3) * R + r]);
                    z = dadd(z, dmul(v0, g0));
                    z = dadd(z, dmul(v1, g1));
                    z = dadd(z, dmul(v2, g2));
                    z = dadd(z, dmul(v3, g3));
                }
                for (; q < e; ++q)
                    z = dadd(z, dmul(static_cast<double>(val[q]),
                                     static_cast<double>(xo[static_cast<int64_t>(col[q]) * R + r])));
                const int64_t ix = static_cast<int64_t>(i) * R + r;
                const double xi = static_cast<double>(xo[ix]);
                if (frozen) {
                    xw[ix] = xo[ix];
                } else {
                    const double xn = cbrt(ddiv(dadd(z, dmul(a, xi)), b));
                    const XT xs = static_cast<XT>(xn);
                    xw[ix] = xs;
                    const double d = dsub(static_cast<double>(xs), xi);
                    const double x2 = dmul(xi, xi);
                    acc[0] = dadd(acc[0], dmul(x2, x2));
                    acc[1] = dadd(acc[1], x2);
                    acc[2] = dadd(acc[2], dmul(xi, z));
                    acc[3] = dadd(acc[3], dmul(d, d));
                }
            }
            restart_sum<R, 4>(acc, red);
            if (threadIdx.x < R && !conv[threadIdx.x]) {
                const double H = dsub(dsub(dmul(ddiv(b, 4.0), acc[0]), dmul(ddiv(a, 2.0), acc[1])),
                                      dmul(0.5, acc[2]));
                const double rr = acc[1] == 0.0 ? 0.0 : ddiv(sqrt(acc[3]), sqrt(acc[1]));
                BatchRestartStat& st = stats[static_cast<int64_t>(k) * R + threadIdx.x];
                st.iters_done = it + 1;
                st.H_last = H;
                st.r_last = rr;
                if (!isfinite(H) || !isfinite(rr)) {
                    st.nonfinite = 1;
                    conv[threadIdx.x] = 1;
                } else if (eps > 0.0 && rr < eps) {
                    st.converged = 1;
                    conv[threadIdx.x] = 1;
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int all = 1;
                for (int q = 0; q < R; ++q) all &= conv[q];
                s_all = all;
            }
            const XT* t = xo;
            xo = xw;
            xw = const_cast<XT*>(t);
            __syncthreads();
            if (s_all) {
                ++it;
                break;
            }
        }
        (void)nonfinite;
        // outputs from the buffer that holds x^(it)
        for (int64_t t = threadIdx.x; t < static_cast<int64_t>(I.n) * R; t += BT) {
            const double v = static_cast<double>(xo[base + t]);
            if (x_out) x_out[base + t] = v;
            if (s_out) s_out[base + t] = v >= 0.0 ? 1 : -1;
        }
        if (threadIdx.x == 0) clock_end[k] = device_clock();
        __syncthreads();
    }
}

// R contiguous iterate entries (one row, all restarts) as one vector access.
template <typename XT, int R>
struct RowVec {
    typedef XT type __attribute__((ext_vector_type(R)));
};
template <typename XT>
struct RowVec<XT, 1> {
    typedef XT type;
};

template <typename XT, int R>
__device__ __forceinline__ void load_row(const XT* p, XT (&out)[R]) {
    const typename RowVec<XT, R>::type w = *reinterpret_cast<const typename RowVec<XT, R>::type*>(p);
    if constexpr (R == 1) {
        out[0] = w;
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) out[r] = w[r];
    }
}

template <typename XT, int R>
__device__ __forceinline__ void store_row(XT* p, const XT (&in)[R]) {
    typename RowVec<XT, R>::type w;
    if constexpr (R == 1) {
        w = in[0];
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = in[r];
    }
    *reinterpret_cast<typename RowVec<XT, R>::type*>(p) = w;
}

// Values other workgroups wrote in the current iteration (partial sums,
// unit flags): agent-scope loads, which miss in this CU's L1.  (A
// workgroup-scope atomic load carries only sc0, which outside
// threadgroup-split dispatches may still hit a stale L1 line.)
__device__ __forceinline__ double ld_coh(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_coh(const int32_t* p) {
    return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int ld_agent(const unsigned int* p) {
    return __hip_atomic_load(const_cast<unsigned int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Which XCD this workgroup runs on (the hardware XCC id register).
__device__ __forceinline__ unsigned int xcd_id() {
    unsigned int v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 0xfu;
}

constexpr unsigned int kStepSpinLimit = 1u << 24;

// Rows [lo, hi) of one instance, restarts [r0, r0 + RJ): z = J x, the
// update of eq:FPE and the sums of eq:Hamilton and Remark S2 (x^4, x^2,
// x z, (dx)^2 per restart).  One row per thread; a coupling costs one index
// and one value (aligned 16-byte chunks, the next chunk requested before
// this one's gathers are waited for) and one contiguous RJ-wide read of the
// iterate (written by the XCD's workgroups in the previous iteration; the
// barrier that ended it invalidated this CU's L1); row sums in ascending
// column order.
template <typename XT, typename VT, int RJ, int WG>
__device__ __forceinline__ void chunk_sweep(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                            const VT* __restrict__ val, int R, int r0, int lo, int hi,
                                            const XT* xo, XT* xw, const bool (&frozen)[RJ], double a, double b,
                                            double (&acc)[4 * RJ]) {
    int sn = 0, en = 0;                 // the next row's offsets, requested early
    if (lo + static_cast<int>(threadIdx.x) < hi) {
        sn = rp[lo + threadIdx.x];
        en = rp[lo + threadIdx.x + 1];
    }
    for (int i = lo + static_cast<int>(threadIdx.x); i < hi; i += WG) {
        const int s = sn, e = en;
        if (i + WG < hi) {
            sn = rp[i + WG];
            en = rp[i + WG + 1];
        }
        double z[RJ];
#pragma unroll
        for (int r = 0; r < RJ; ++r) z[r] = 0.0;
        using CV = typename Vec4<int>::type;
        using VV = typename Vec4<VT>::type;
        int c0 = s & ~3;
        CV cn{};
        VV vn{};
        if (c0 < e) {
            cn = *reinterpret_cast<const CV*>(col + c0);
            vn = *reinterpret_cast<const VV*>(val + c0);
        }
        for (; c0 < e; c0 += 4) {
            const CV cv = cn;
            const VV vv = vn;
            if (c0 + 4 < e) {
                cn = *reinterpret_cast<const CV*>(col + c0 + 4);
                vn = *reinterpret_cast<const VV*>(val + c0 + 4);
            }
            const int cc[4] = {cv.x, cv.y, cv.z, cv.w};
            const double vd[4] = {static_cast<double>(vv.x), static_cast<double>(vv.y),
                                  static_cast<double>(vv.z), static_cast<double>(vv.w)};
            XT g[4][RJ];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c0 + u >= s && c0 + u < e) load_row<XT, RJ>(xo + static_cast<int64_t>(cc[u]) * R + r0, g[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c0 + u >= s && c0 + u < e) {
#pragma unroll
                    for (int r = 0; r < RJ; ++r) z[r] = dadd(z[r], dmul(vd[u], static_cast<double>(g[u][r])));
                }
        }
        XT xi[RJ], xn[RJ];
        load_row<XT, RJ>(xo + static_cast<int64_t>(i) * R + r0, xi);
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
            const double xv = static_cast<double>(xi[r]);
            if (frozen[r]) {
                xn[r] = xi[r];
            } else {
                xn[r] = static_cast<XT>(cbrt(ddiv(dadd(z[r], dmul(a, xv)), b)));
                const double d = dsub(static_cast<double>(xn[r]), xv);
                const double x2 = dmul(xv, xv);
                acc[4 * r + 0] = dadd(acc[4 * r + 0], dmul(x2, x2));
                acc[4 * r + 1] = dadd(acc[4 * r + 1], x2);
                acc[4 * r + 2] = dadd(acc[4 * r + 2], dmul(xv, z[r]));
                acc[4 * r + 3] = dadd(acc[4 * r + 3], dmul(d, d));
            }
        }
        store_row<XT, RJ>(xw + static_cast<int64_t>(i) * R + r0, xn);
    }
}

// Barrier `target` of the workgroups counted on *bar (all on one XCD, or
// the whole grid at launch): every wave waits for its stores to reach the
// XCD's L2, thread 0 counts the workgroup in and polls, and afterwards an
// agent-scope acquire invalidates this CU's L1, so that plain loads see
// what the XCD's workgroups wrote before the barrier.  Returns false if the
// wait exceeded its bound or another workgroup gave up (the abort word is
// then set and the caller leaves the kernel).
__device__ __forceinline__ bool counter_barrier(unsigned int* bar, unsigned int target, unsigned int* abort_word,
                                                int* s_flag) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned int spins = 0;
        int ok = 1;
        while (ld_agent(bar) < target) {
            if (++spins > kStepSpinLimit || ld_agent(abort_word) != 0u) {
                __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *s_flag = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *s_flag != 0;
}

// The batch loop for up to 8 restarts: every XCD iterates its share of the
// units (restart groups of instances) in lockstep.  The host deals the
// units to the XCDs by work and cuts each unit's rows into chunks; the
// chunks of an XCD go round-robin to the workgroups running on it (ranks
// taken at launch from the hardware XCD id), so every instance is spread
// over all of them and a unit that stops takes the same share of work from
// each.  Iteration k: every workgroup sweeps its chunks of running units
// (reading x^(k) from L2, where the XCD's workgroups wrote it) and stores
// the chunk's partial sums; the workgroup that completes a unit's count of
// chunks adds the unit's partials in chunk order, takes the stopping
// decisions of Remark S2 for its restarts (a stopped restart is copied
// forward from then on) and marks the unit done when all stopped or after
// max_iters iterations; then the XCD's workgroups meet at a barrier.  An
// XCD leaves the loop once all its units are done.  No XCD waits for
// another.  A unit's time to solution is the clock when it was marked done.
template <typename XT, typename VT, int RJ, int WG>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(RJ >= 8 ? 2 : RJ >= 4 ? 3 : 4))) void batch_step_kernel(const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const VT* __restrict__ val, XT* xa, XT* xb,
                                                        const BatchStepArgs* __restrict__ args) {
    constexpr int K = 4 * RJ;                 // x^4, x^2, x z, (dx)^2 per restart
    constexpr int NW = WG / kWave;
    constexpr int SPLIT = WG / K;             // threads per quantity in a unit's reduction
    __shared__ double red[K * NW];
    __shared__ double tot[K * SPLIT];
    __shared__ int s_rank, s_w, s_flag, s_last, s_done;
    const BatchStepArgs& A = *args;
    const BatchPlan& pl = A.plan;
    const int R = A.R;
    unsigned int* ctr = pl.counters;
    unsigned int* abort_word = ctr + 32 * 25;
    const unsigned int x = xcd_id() % static_cast<unsigned int>(pl.n_xcd);
    if (threadIdx.x == 0) {
        atomicMin(reinterpret_cast<unsigned long long*>(A.clock_start),
                  static_cast<unsigned long long>(device_clock()));
        s_rank = static_cast<int>(__hip_atomic_fetch_add(ctr + 32 * x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    // every workgroup registered once: the ranks are final after this
    if (!counter_barrier(ctr + 32 * 24, gridDim.x, abort_word, &s_flag)) return;
    if (threadIdx.x == 0) {
        s_w = static_cast<int>(ld_agent(ctr + 32 * x));
        // an XCD without workgroups would leave its units unrun
        if (blockIdx.x == 0)
            for (int q = 0; q < pl.n_xcd; ++q)
                if (ld_agent(ctr + 32 * q) == 0u) __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int rank = s_rank, W = s_w;
    const int c_lo = pl.off[x], c_hi = pl.off[x + 1];
    const int my_units = pl.units_on[x];
    unsigned int* bar = ctr + 32 * (8 + x);
    unsigned int* ndone = ctr + 32 * (16 + x);
    // x^(0) into buffer a for this workgroup's chunks
    for (int c = c_lo + rank; c < c_hi; c += W) {
        const BatchChunk ch = pl.chunks[c];
        const int r0 = pl.units[ch.unit].r0;
        for (int64_t t = threadIdx.x; t < static_cast<int64_t>(ch.hi - ch.lo) * RJ; t += WG) {
            const int64_t e = (ch.lo + t / RJ) * static_cast<int64_t>(R) + r0 + t % RJ;
            xa[e] = static_cast<XT>(A.x0[e]);
        }
    }
    unsigned int gen = 1;
    if (!counter_barrier(bar, W * gen, abort_word, &s_flag)) return;
    for (int64_t it = 0; it < A.max_iters; ++it) {
        const XT* xo = (it & 1) ? xb : xa;
        XT* xw = (it & 1) ? xa : xb;
        for (int c = c_lo + rank; c < c_hi; c += W) {
            const BatchChunk ch = pl.chunks[c];
            const int u = ch.unit;
            // a unit's flags change only after all its chunks of the
            // iteration are done, and were last written before the barrier
            // that began it (which invalidated L1): plain loads see them
            if (pl.done[u] != 0) continue;
            const BatchUnit U = pl.units[u];
            const int k = U.inst;
            const double a = A.alpha[k], b = A.beta[k];
            bool frozen[RJ];
#pragma unroll
            for (int r = 0; r < RJ; ++r) frozen[r] = pl.conv[static_cast<int64_t>(u) * RJ + r] != 0;
            double acc[K];
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] = 0.0;
            chunk_sweep<XT, VT, RJ, WG>(rp, col, val, R, U.r0, ch.lo, ch.hi, xo, xw, frozen, a, b, acc);
            block_sum<K, WG>(acc, red);       // the chunk's totals in thread 0
            if (threadIdx.x == 0) {
                double* p = pl.partials + static_cast<size_t>(ch.slot) * K;
#pragma unroll
                for (int q = 0; q < K; ++q) p[q] = acc[q];
                s_last = arrive_last(pl.tickets + 32 * static_cast<size_t>(u), static_cast<unsigned int>(U.nchunks));
            }
            __syncthreads();
            if (!s_last) continue;
            // the unit's last chunk: its partials in chunk order (thread
            // (q, j) adds chunks j, j + SPLIT, ... of quantity q; then the
            // SPLIT sums in order)
            {
                const int q = threadIdx.x % K, j0 = threadIdx.x / K;
                double v = 0.0;
                if (j0 < SPLIT)
                    for (int j = j0; j < U.nchunks; j += SPLIT)
                        v = dadd(v, ld_coh(pl.partials + (static_cast<size_t>(U.first_slot) + j) * K + q));
                if (j0 < SPLIT) tot[j0 * K + q] = v;
            }
            __syncthreads();
            if (threadIdx.x < RJ) {
                const int r = threadIdx.x;
                double S[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    double v = 0.0;
                    for (int j = 0; j < SPLIT; ++j) v = dadd(v, tot[j * K + 4 * r + m]);
                    S[m] = v;
                }
                int32_t* cv = pl.conv + static_cast<int64_t>(u) * RJ + r;
                if (!frozen[r]) {
                    const double H = dsub(dsub(dmul(ddiv(b, 4.0), S[0]), dmul(ddiv(a, 2.0), S[1])), dmul(0.5, S[2]));
                    const double rr = S[1] == 0.0 ? 0.0 : ddiv(sqrt(S[3]), sqrt(S[1]));
                    BatchRestartStat& st = A.stats[static_cast<int64_t>(k) * R + U.r0 + r];
                    st.iters_done = it + 1;
                    st.H_last = H;
                    st.r_last = rr;
                    if (!isfinite(H) || !isfinite(rr)) {
                        st.nonfinite = 1;
                        *cv = 1;
                    } else if (A.eps > 0.0 && rr < A.eps) {
                        st.converged = 1;
                        *cv = 1;
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int all = 1;
                for (int r = 0; r < RJ; ++r) all &= ld_coh(pl.conv + static_cast<int64_t>(u) * RJ + r) != 0;
                if (all || it + 1 == A.max_iters) {
                    pl.done[u] = static_cast<int32_t>(it + 1);
                    atomicMax(reinterpret_cast<unsigned long long*>(A.clock_end + k),
                              static_cast<unsigned long long>(device_clock()));
                    __hip_atomic_fetch_add(ndone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                reset_ticket(pl.tickets + 32 * static_cast<size_t>(u));
            }
        }
        ++gen;
        if (!counter_barrier(bar, W * gen, abort_word, &s_flag)) return;
        if (threadIdx.x == 0) s_done = static_cast<int>(ld_agent(ndone)) >= my_units;
        __syncthreads();
        if (s_done) break;
    }
    // outputs of this workgroup's chunks, from the buffer of each unit's last iterate
    for (int c = c_lo + rank; c < c_hi; c += W) {
        const BatchChunk ch = pl.chunks[c];
        const int r0 = pl.units[ch.unit].r0;
        const XT* xf = (ld_coh(pl.done + ch.unit) & 1) ? xb : xa;
        for (int64_t t = threadIdx.x; t < static_cast<int64_t>(ch.hi - ch.lo) * RJ; t += WG) {
            const int64_t e = (ch.lo + t / RJ) * static_cast<int64_t>(R) + r0 + t % RJ;
            const double v = static_cast<double>(xf[e]);
            if (A.x_out) A.x_out[e] = v;
            if (A.s_out) A.s_out[e] = v >= 0.0 ? 1 : -1;
        }
    }
}

template <int R>
__global__ void batch_init_kernel(BatchRestartStat* stats, int count, unsigned int* queue,
                                  uint64_t* clock_start, uint64_t* clock_end, unsigned int* counters,
                                  unsigned int* tickets, int32_t* done, int32_t* conv, int n_units, int rj) {
    const int64_t total = static_cast<int64_t>(count) * R;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t t = t0; t < count; t += stride) clock_end[t] = 0;
    for (int64_t t = t0; t < total; t += stride) {
        stats[t].iters_done = 0;
        stats[t].converged = 0;
        stats[t].nonfinite = 0;
        stats[t].H_last = 0.0;
        stats[t].r_last = 0.0;
    }
    if (counters) {
        for (int64_t t = t0; t < kBatchCounterWords; t += stride) counters[t] = 0u;
        for (int64_t t = t0; t < static_cast<int64_t>(n_units) * 32; t += stride) tickets[t] = 0u;
        for (int64_t t = t0; t < n_units; t += stride) done[t] = 0;
        for (int64_t t = t0; t < static_cast<int64_t>(n_units) * rj; t += stride) conv[t] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *queue = 0u;
        *clock_start = ~0ull;
    }
}

// eq:IsingModel per instance and restart (workgroup per instance).
template <typename VT, int R>
__global__ __launch_bounds__(BT) void batch_energy_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const VT* __restrict__ val,
    const BatchInstance* __restrict__ inst, int count, const int8_t* __restrict__ s,
    int want_int, double* __restrict__ E, int64_t* __restrict__ E_int) {
    constexpr int S = BT / R;
    __shared__ double red[BW * R];
    const int r = threadIdx.x % R;
    const int slot = threadIdx.x / R;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const BatchInstance I = inst[k];
        double eJ = 0.0;
        int64_t eI = 0;
        for (int i = I.row0 + slot; i < I.row0 + I.n; i += S) {
            double acc = 0.0;
            int64_t iacc = 0;
            for (int q = rp[i]; q < rp[i + 1]; ++q) {
                const double sj = static_cast<double>(s[static_cast<int64_t>(col[q]) * R + r]);
                const double v = static_cast<double>(val[q]);
                acc = dadd(acc, dmul(v, sj));
                if (want_int) iacc += static_cast<int64_t>(v) * static_cast<int64_t>(sj);
            }
            const double si = static_cast<double>(s[static_cast<int64_t>(i) * R + r]);
            eJ = dadd(eJ, dmul(si, acc));
            eI += static_cast<int64_t>(si) * iacc;
        }
        // the int64 sum travels exactly as two doubles (high and low 32 bits)
        double v[1] = {eJ};
        restart_sum<R, 1>(v, red);
        double hi[1] = {static_cast<double>(eI >> 32)};
        double lo[1] = {static_cast<double>(eI & 0xffffffffLL)};
        restart_sum<R, 1>(hi, red);
        restart_sum<R, 1>(lo, red);
        if (threadIdx.x < R) {
            const int64_t tot = static_cast<int64_t>(hi[0]) * 4294967296LL + static_cast<int64_t>(lo[0]);
            if (E) E[static_cast<int64_t>(k) * R + threadIdx.x] = dmul(-0.5, v[0]);
            if (E_int) E_int[static_cast<int64_t>(k) * R + threadIdx.x] = -(tot / 2);
        }
        __syncthreads();
    }
}

// Per-instance matrix statistics for eq:alphabeta (workgroup per instance):
// out[k] = {max_i sum_j |J_ij|, sum J_ij, #stored, sum (J_ij - mean)^2}.
template <typename VT>
__global__ __launch_bounds__(BT) void batch_stats_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const VT* __restrict__ val,
    const BatchInstance* __restrict__ inst, int count, double* __restrict__ out) {
    __shared__ double red[3 * BW];
    __shared__ double redm[BW];
    __shared__ double s_mean;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const BatchInstance I = inst[k];
        double v[3] = {0.0, 0.0, 0.0};
        double pmax = 0.0;
        for (int i = I.row0 + threadIdx.x; i < I.row0 + I.n; i += BT) {
            double rs = 0.0;
            for (int q = rp[i]; q < rp[i + 1]; ++q) {
                if (col[q] == i) continue;
                const double x = static_cast<double>(val[q]);
                rs = dadd(rs, fabs(x));
                v[0] = dadd(v[0], x);
                v[1] += 1.0;
            }
            pmax = fmax(pmax, rs);
        }
        double v2[2] = {v[0], v[1]};
        block_sum<2, BT>(v2, red);
        v[0] = v2[0];
        v[1] = v2[1];
        const double wm = wave_max(pmax);
        if ((threadIdx.x & (kWave - 1)) == 0) redm[threadIdx.x / kWave] = wm;
        __syncthreads();
        const double nn = static_cast<double>(I.n);
        if (threadIdx.x == 0) {
            double m = 0.0;
            for (int w = 0; w < BW; ++w) m = fmax(m, redm[w]);
            out[4 * k + 0] = m;
            out[4 * k + 1] = v[0];
            out[4 * k + 2] = v[1];
            s_mean = nn > 1.0 ? v[0] / (nn * (nn - 1.0)) : 0.0;
        }
        __syncthreads();
        const double mean = s_mean;
        double ss[1] = {0.0};
        for (int i = I.row0 + threadIdx.x; i < I.row0 + I.n; i += BT)
            for (int q = rp[i]; q < rp[i + 1]; ++q) {
                if (col[q] == i) continue;
                const double d = dsub(static_cast<double>(val[q]), mean);
                ss[0] = dadd(ss[0], dmul(d, d));
            }
        block_sum<1, BT>(ss, red);
        if (threadIdx.x == 0) out[4 * k + 3] = ss[0];
        __syncthreads();
    }
}

// lambda_max(-J) of each selected instance by power iteration on cI - J
// (workgroup per instance, no host round trips).  v and w are scratch of the
// batch's total row count; lam[k] receives mu - c.
template <typename VT>
__global__ __launch_bounds__(BT) void batch_power_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const VT* __restrict__ val,
    const BatchInstance* __restrict__ inst, const int32_t* __restrict__ jobs, int njobs,
    const double* __restrict__ cshift, double tol, int64_t maxit, double* __restrict__ v,
    double* __restrict__ w, double* __restrict__ lam) {
    __shared__ double red[2 * BW];
    __shared__ double s_bcast[2];
    for (int jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
        const int k = jobs[jb];
        const BatchInstance I = inst[k];
        const double c = cshift[k];
        // start vector: a fixed SplitMix64 sequence, normalised
        double nrm[1] = {0.0};
        for (int i = threadIdx.x; i < I.n; i += BT) {
            uint64_t q = 0x9E3779B97F4A7C15ULL * static_cast<uint64_t>(i + 1);
            q = (q ^ (q >> 30)) * 0xBF58476D1CE4E5B9ULL;
            q = (q ^ (q >> 27)) * 0x94D049BB133111EBULL;
            q ^= q >> 31;
            const double u = 2.0 * (static_cast<double>(q >> 11) * 0x1.0p-53) - 1.0;
            v[I.row0 + i] = u;
            nrm[0] = dadd(nrm[0], dmul(u, u));
        }
        block_sum<1, BT>(nrm, red);
        if (threadIdx.x == 0) s_bcast[0] = sqrt(nrm[0]);
        __syncthreads();
        const double n0 = s_bcast[0];
        for (int i = threadIdx.x; i < I.n; i += BT) v[I.row0 + i] = ddiv(v[I.row0 + i], n0);
        __syncthreads();
        double mu = 0.0, mu_prev = 0.0;
        for (int64_t it = 0; it < maxit; ++it) {
            double acc[2] = {0.0, 0.0};
            for (int i = I.row0 + threadIdx.x; i < I.row0 + I.n; i += BT) {
                double z = 0.0;
                for (int q = rp[i]; q < rp[i + 1]; ++q)
                    z = dadd(z, dmul(static_cast<double>(val[q]), v[col[q]]));
                const double wi = dsub(dmul(c, v[i]), z);
                w[i] = wi;
                acc[0] = dadd(acc[0], dmul(v[i], wi));
                acc[1] = dadd(acc[1], dmul(wi, wi));
            }
            block_sum<2, BT>(acc, red);
            if (threadIdx.x == 0) {
                s_bcast[0] = acc[0];
                s_bcast[1] = sqrt(acc[1]);
            }
            __syncthreads();
            mu = s_bcast[0];
            const double wn = s_bcast[1];
            if (wn == 0.0) break;
            for (int i = I.row0 + threadIdx.x; i < I.row0 + I.n; i += BT) v[i] = ddiv(w[i], wn);
            __syncthreads();
            if (it > 0 && fabs(mu - mu_prev) <= tol * fabs(mu)) break;
            mu_prev = mu;
        }
        if (threadIdx.x == 0) lam[k] = mu - c;
        __syncthreads();
    }
}

// Every coupling of a row must stay inside its instance's diagonal block.
__global__ __launch_bounds__(256) void batch_validate_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const BatchInstance* __restrict__ inst, int count, int64_t n, int32_t* bad) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {                      // last instance with row0 <= i
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].row0 <= i) lo = mid; else hi = mid - 1;
        }
        const int a = inst[lo].row0, b = inst[lo].row0 + inst[lo].n;
        for (int q = rp[i]; q < rp[i + 1]; ++q)
            if (col[q] < a || col[q] >= b) atomicOr(bad, 1);
    }
}

template <typename T>
int resident_grid(T kern, int threads) {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, 0) != hipSuccess || occ < 1) occ = 1;
    return cus * occ;
}

}  // namespace

#define DOCH_BATCH_R(R, ...)                                  \
    switch (R) {                                              \
        case 1: { constexpr int RR = 1; __VA_ARGS__; } break;  \
        case 2: { constexpr int RR = 2; __VA_ARGS__; } break;  \
        case 4: { constexpr int RR = 4; __VA_ARGS__; } break;  \
        case 8: { constexpr int RR = 8; __VA_ARGS__; } break;  \
        case 16: { constexpr int RR = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int RR = 32; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                 \
    }

bool batch_restarts_supported(int R) {
    return R == 1 || R == 2 || R == 4 || R == 8 || R == 16 || R == 32;
}

// The (restarts per unit, threads) pairs the lockstep kernel is built for.
static bool step_shape_built(int rj, int wg) {
    switch (rj) {
        case 8:
        case 4: return wg == 256 || wg == 512;
        case 2:
        case 1: return wg == 512 || wg == 1024;
        default: return false;
    }
}

bool batch_shape_supported(const BatchShape& sh, int R) {
    if (R > 8) return true;                   // restart-per-lane kernel, no shape
    if (sh.chunk_rows < 1) return false;
    if (sh.rj != 1 && sh.rj != 2 && sh.rj != 4 && sh.rj != 8) return false;
    return step_shape_built(std::min(sh.rj, R), sh.wg);
}

// Calls f(kernel pointer, WG tag) for the lockstep kernel of the shape.
template <typename XT, typename VT, typename F>
static hipError_t with_step_kernel(int RJ, int WG, F&& f) {
    using std::integral_constant;
#define DOCH_STEP(RJV, WGV)                                                                          \
    if (RJ == RJV && WG == WGV)                                                                      \
        return f(batch_step_kernel<XT, VT, RJV, WGV>, integral_constant<int, WGV>());
    DOCH_STEP(8, 256)
    DOCH_STEP(8, 512)
    DOCH_STEP(4, 256)
    DOCH_STEP(4, 512)
    DOCH_STEP(2, 512)
    DOCH_STEP(2, 1024)
    DOCH_STEP(1, 512)
    DOCH_STEP(1, 1024)
#undef DOCH_STEP
    return hipErrorInvalidValue;
}

template <typename F>
static hipError_t with_types(int x_dtype, int vt, F&& f) {
    if (vt == ISING_F64) return x_dtype == ISING_F64 ? f(double(), double()) : f(float(), double());
    return x_dtype == ISING_F64 ? f(double(), float()) : f(float(), float());
}

int batch_shape_grid(const BatchShape& sh, int x_dtype, int vt) {
    int grid = 0;
    (void)with_types(x_dtype, vt, [&](auto xtag, auto vtag) {
        using XT = decltype(xtag);
        using VT = decltype(vtag);
        return with_step_kernel<XT, VT>(sh.rj, sh.wg, [&](auto kern, auto wgtag) {
            grid = resident_grid(kern, decltype(wgtag)::value);
            return hipSuccess;
        });
    });
    return grid;
}

hipError_t launch_batch_solve(const BatchView& B, int R, const BatchShape& shape, const BatchPlan& plan,
                              const BatchStepArgs* args_dev, int64_t max_iters, const double* alpha,
                              const double* beta, double eps, int x_dtype, const double* x0,
                              void* xa, void* xb, unsigned int* queue, BatchRestartStat* stats,
                              uint64_t* clock_start, uint64_t* clock_end, double* x_out,
                              int8_t* s_out, hipStream_t s) {
    if (!batch_restarts_supported(R)) return hipErrorInvalidValue;
    const int ig = static_cast<int>(std::min<int64_t>(1024, (static_cast<int64_t>(B.count) * R + 255) / 256));
    const bool lockstep = R <= 8;
    DOCH_BATCH_R(R, {
        hipLaunchKernelGGL(batch_init_kernel<RR>, dim3(ig), dim3(256), 0, s, stats, B.count, queue,
                           clock_start, clock_end, lockstep ? plan.counters : nullptr, plan.tickets, plan.done,
                           plan.conv, lockstep ? plan.n_units : 0, plan.rj);
    });
    if (lockstep) {
        if (!batch_shape_supported(shape, R)) return hipErrorInvalidValue;
        hipError_t e = with_types(x_dtype, B.vt, [&](auto xtag, auto vtag) {
            using XT = decltype(xtag);
            using VT = decltype(vtag);
            return with_step_kernel<XT, VT>(std::min(shape.rj, R), shape.wg, [&](auto kern, auto wgtag) {
                constexpr int WG = decltype(wgtag)::value;
                hipLaunchKernelGGL(kern, dim3(resident_grid(kern, WG)), dim3(WG), 0, s, B.rp, B.col,
                                   static_cast<const VT*>(B.val), static_cast<XT*>(xa), static_cast<XT*>(xb), args_dev);
                return hipSuccess;
            });
        });
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    DOCH_BATCH_R(R, {
        if constexpr (RR > 8) {
            auto go = [&](auto xtag, auto vtag) {
                using XT = decltype(xtag);
                using VT = decltype(vtag);
                auto kern = batch_solve_kernel<XT, VT, RR>;
                const int grid = std::min(resident_grid(kern, BT), B.count);
                hipLaunchKernelGGL(kern, dim3(grid), dim3(BT), 0, s, B.rp, B.col, static_cast<const VT*>(B.val),
                                   B.inst, B.order, B.count, alpha, beta, eps, max_iters, x0,
                                   static_cast<XT*>(xa), static_cast<XT*>(xb), queue, stats, clock_start,
                                   clock_end, x_out, s_out);
                return hipSuccess;
            };
            (void)with_types(x_dtype, B.vt, go);
        }
    });
    return hipGetLastError();
}

hipError_t launch_batch_validate(const BatchView& B, int64_t n, int32_t* bad, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(batch_validate_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, B.rp,
                       B.col, B.inst, B.count, n, bad);
    return hipGetLastError();
}

hipError_t launch_batch_energy(const BatchView& B, const int8_t* s_spins, int R, double* E,
                               int64_t* E_int, hipStream_t s) {
    const int grid = std::min(B.count, 2048);
    DOCH_BATCH_R(R, {
        if (B.vt == ISING_F64)
            hipLaunchKernelGGL((batch_energy_kernel<double, RR>), dim3(grid), dim3(BT), 0, s, B.rp,
                               B.col, static_cast<const double*>(B.val), B.inst, B.count, s_spins,
                               E_int != nullptr, E, E_int);
        else
            hipLaunchKernelGGL((batch_energy_kernel<float, RR>), dim3(grid), dim3(BT), 0, s, B.rp,
                               B.col, static_cast<const float*>(B.val), B.inst, B.count, s_spins,
                               E_int != nullptr, E, E_int);
    });
    return hipGetLastError();
}

hipError_t launch_batch_stats(const BatchView& B, double* out, hipStream_t s) {
    const int grid = std::min(B.count, 2048);
    if (B.vt == ISING_F64)
        hipLaunchKernelGGL(batch_stats_kernel<double>, dim3(grid), dim3(BT), 0, s, B.rp, B.col,
                           static_cast<const double*>(B.val), B.inst, B.count, out);
    else
        hipLaunchKernelGGL(batch_stats_kernel<float>, dim3(grid), dim3(BT), 0, s, B.rp, B.col,
                           static_cast<const float*>(B.val), B.inst, B.count, out);
    return hipGetLastError();
}

hipError_t launch_batch_power(const BatchView& B, const int32_t* jobs, int njobs,
                              const double* cshift, double tol, int64_t maxit, double* v, double* w,
                              double* lam, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    const int grid = std::min(njobs, 2048);
    if (B.vt == ISING_F64)
        hipLaunchKernelGGL(batch_power_kernel<double>, dim3(grid), dim3(BT), 0, s, B.rp, B.col,
                           static_cast<const double*>(B.val), B.inst, jobs, njobs, cshift, tol,
                           maxit, v, w, lam);
    else
        hipLaunchKernelGGL(batch_power_kernel<float>, dim3(grid), dim3(BT), 0, s, B.rp, B.col,
                           static_cast<const float*>(B.val), B.inst, jobs, njobs, cshift, tol,
                           maxit, v, w, lam);
    return hipGetLastError();
}

}  // namespace doch
