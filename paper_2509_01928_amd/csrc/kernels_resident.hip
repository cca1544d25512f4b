// kernels_resident.hip -- a whole single-restart DOCH run (Alg. 1, eq:FPE,
// eq:Hamilton, Remark S2) in one cooperative launch, for problems small
// enough that launching a kernel per iteration costs more than the
// iteration itself.
//
// Workgroups 0..G-1 own rows; workgroup G is the reducer.  Iteration k:
//   1. each row workgroup reads x^(k) at the device's point of coherence
//      (the iterate crosses XCDs, whose L2 caches are not coherent with each
//      other), forms its rows of Jhat x^(k), applies the cube-root update and
//      writes x^(k+1) the same way; its partial sums go to one of two
//      partial buffers (iterations alternate);
//   2. the reducer meanwhile finishes H(x^(k-1)) and r^(k-1) from the other
//      buffer, logs them and, on convergence or a non-finite value, publishes
//      a stop that every workgroup sees at the next barrier;
//   3. grid barrier k+1: two-level arrival counters (one per XCD group, then
//      one for the groups) and one release word per group;
//   4. with a field, every workgroup adds the h x partials of iteration k in
//      the same fixed order and forms the extra spin t^(k+1) itself.
// Because the stop is seen one iteration late, the iterate rotates through
// three buffers: x^(k) survives the iteration that runs before the stop is
// seen.  J, the field and the row offsets are read-only for the whole launch
// and stay in the L2 caches (dense rows of up to 2048 entries live in
// registers).  Every row is summed in ascending column order exactly as in
// the per-iteration kernels, so the iterates are bit-identical to theirs.
//
// Every wait is bounded: a workgroup that polls for more than a few seconds
// marks the run as timed out and publishes the stop, so every wave exits.
#include "device_common.h"
#include "ising_internal.h"
#include "step_common.h"

namespace doch {

static_assert(kTicketStride == 32, "ResidentSync spaces its counters one 128-byte line apart");

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;
constexpr unsigned int kSpinLimit = 1u << 22;

template <typename T>
__device__ __forceinline__ T ld_coh(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int add_coh(unsigned int* p, unsigned int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish a stop on every group's release word (upper half).
__device__ void publish_stop(ResidentSync* sy, unsigned int groups, unsigned int why) {
    for (unsigned int q = 0; q < groups; ++q) st_coh(&sy->flag[q * kTicketStride + 1], why);
}

// Grid barrier number `gen` (1, 2, ...).  Every wave first waits for its own
// stores (the iterate, the partials) to complete (both counters: a store
// through a generic pointer counts in each); thread 0 then counts the
// workgroup in and polls its group's release word, whose lower half is the
// last released barrier and upper half a published stop.  Returns false when
// the run stops.
__device__ bool grid_barrier(ResidentSync* sy, unsigned int gen, RestartState* st) {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();
    __shared__ int go;
    if (threadIdx.x == 0) {
        const unsigned int G = gridDim.x;
        const unsigned int g = blockIdx.x & 7u;
        const unsigned int per = (G - g + 7u) / 8u;
        const unsigned int groups = G < 8u ? G : 8u;
        if (add_coh(&sy->grp[g * kTicketStride], 1u) == gen * per - 1u) {
            if (add_coh(&sy->top[0], 1u) == gen * groups - 1u)
                for (unsigned int q = 0; q < groups; ++q) st_coh(&sy->flag[q * kTicketStride], gen);
        }
        const unsigned long long* f =
            reinterpret_cast<const unsigned long long*>(sy->flag + g * kTicketStride);
        unsigned int spins = 0;
        int ok = 1;
        for (;;) {
            const unsigned long long v = ld_coh(f);
            if (static_cast<unsigned int>(v >> 32) != 0u) { ok = 0; break; }
            if (static_cast<unsigned int>(v) >= gen) break;
            if (++spins > kSpinLimit) {
                st_coh(&st->aborted, 1);
                st_coh(&st->done, 1);
                publish_stop(sy, groups, 2u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        go = ok;
    }
    __syncthreads();
    return go != 0;
}

// Sum quantity q of the G row workgroups' partials in a fixed order (thread
// t takes workgroups t, t + NT, ...; then the workgroup sum), the same in
// every workgroup that calls it.  Valid in thread 0.
template <int NQ>
__device__ void sum_partials(const double* __restrict__ p, int G, const int (&qs)[NQ], double (&out)[NQ],
                             double* lds) {
#pragma unroll
    for (int j = 0; j < NQ; ++j) out[j] = 0.0;
    for (int g0 = 0; g0 < G; g0 += 4 * NT) {
        double v[4][NQ];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int g = g0 + b * NT + static_cast<int>(threadIdx.x);
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                v[b][j] = g < G ? ld_coh(p + static_cast<size_t>(g) * kNumPartials + qs[j]) : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int j = 0; j < NQ; ++j) out[j] = dadd(out[j], v[b][j]);
    }
    block_sum<NQ, NT>(out, lds);
}

// t^(k+1) = cbrt((z_n + alpha t^(k)) / beta) with z_n = sum_i h_i x_i^(k),
// rounded to the iterate's storage type; identical in every workgroup.
template <typename XT>
__device__ double next_t(const double* p, int G, double t, const ResidentArgs& a, double* lds,
                         double* zn_out) {
    __shared__ double tb[2];
    const int qs[1] = {P_HX};
    double s[1];
    sum_partials<1>(p, G, qs, s, lds);
    if (threadIdx.x == 0) {
        const double zn = s[0];
        const XT ts = static_cast<XT>(cbrt(ddiv(dadd(zn, dmul(a.alpha, t)), a.beta)));
        tb[0] = static_cast<double>(ts);
        tb[1] = zn;
    }
    __syncthreads();
    const double tn = tb[0];
    if (zn_out) *zn_out = tb[1];
    __syncthreads();
    return tn;
}

// The reducer's work for iteration j: H(x^(j)), r^(j), the log, the state
// and, if the run ends here, the stop.
template <typename XT, bool FIELD>
__device__ void finish_iteration(const ResidentArgs& a, int64_t j, const double* p, double t,
                                 double* lds) {
    const int qs[4] = {P_X4, P_X2, P_XZ, P_DX2};
    double s[4];
    sum_partials<4>(p, a.row_groups, qs, s, lds);
    double zn = 0.0, tn = 0.0;
    if (FIELD) tn = next_t<XT>(p, a.row_groups, t, a, lds, &zn);
    if (threadIdx.x != 0) return;
    double S4 = s[0], S2 = s[1], Sxz = s[2], Sd = s[3];
    if (FIELD) {
        const double t2 = dmul(t, t);
        S4 = dadd(S4, dmul(t2, t2));
        S2 = dadd(S2, t2);
        Sxz = dadd(Sxz, dmul(t, zn));
        const double d = dsub(tn, t);
        Sd = dadd(Sd, dmul(d, d));
    }
    const double H = dsub(dsub(dmul(ddiv(a.beta, 4.0), S4), dmul(ddiv(a.alpha, 2.0), S2)), dmul(0.5, Sxz));
    const double r = (S2 == 0.0) ? 0.0 : ddiv(sqrt(Sd), sqrt(S2));
    a.log[2 * j] = H;
    a.log[2 * j + 1] = r;
    RestartState* st = a.state;
    st->iters_done = j + 1;
    st->H_last = H;
    st->r_last = r;
    bool stop = false;
    if (!isfinite(H) || !isfinite(r)) {
        st->nonfinite = 1;
        stop = true;
    } else if (a.eps > 0.0 && r < a.eps) {
        st->converged = 1;
        stop = true;
    }
    if (stop) {
        st->done = 1;
        const unsigned int G = gridDim.x;
        publish_stop(a.sync, G < 8u ? G : 8u, 1u);
    }
}

// The iteration loop shared by the dense and sparse kernels.  rows(xo, xn,
// t, acc) does this workgroup's rows of one iteration.
template <typename XT, bool FIELD, typename Rows>
__device__ void resident_loop(const ResidentArgs& a, int64_t n, const Rows& rows) {
    __shared__ double red[kNumPartials * NW];
    XT* const xbase = static_cast<XT*>(a.x);
    auto xb = [&](int64_t b) { return xbase + b * a.xstride; };   // buffer b of 3
    const int G = a.row_groups;
    const bool reducer = static_cast<int>(blockIdx.x) == G;
    double t = FIELD ? static_cast<double>(ld_coh(xb(0) + n)) : 0.0;   // t^(k)
    double t_prev = t;                                                  // t^(k-1)
    for (int64_t k = 0; k < a.iters; ++k) {
        double* pk = a.partials + static_cast<size_t>(k & 1) * G * kNumPartials;
        if (!reducer) {
            double acc[kNumPartials];
#pragma unroll
            for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;
            rows(xb(k % 3), xb((k + 1) % 3), t, acc);
            block_sum<kNumPartials, NT>(acc, red);
            if (threadIdx.x == 0)
#pragma unroll
                for (int q = 0; q < kNumPartials; ++q) store_agent(pk + static_cast<size_t>(blockIdx.x) * kNumPartials + q, acc[q]);
        } else if (k > 0) {
            finish_iteration<XT, FIELD>(a, k - 1, a.partials + static_cast<size_t>((k - 1) & 1) * G * kNumPartials,
                                        t_prev, red);
        }
        if (!grid_barrier(a.sync, static_cast<unsigned int>(k + 1), a.state)) return;
        if (FIELD) {
            t_prev = t;
            t = next_t<XT>(pk, G, t, a, red, nullptr);
            if (blockIdx.x == 0 && threadIdx.x == 0) st_coh(xb((k + 1) % 3) + n, static_cast<XT>(t));
        } else {
            t_prev = t;
        }
    }
    if (reducer && a.iters > 0)
        finish_iteration<XT, FIELD>(a, a.iters - 1,
                                    a.partials + static_cast<size_t>((a.iters - 1) & 1) * G * kNumPartials, t_prev,
                                    red);
}

// Row i's update from z = (Jhat x^(k))_i: store x^(k+1)_i at the point of
// coherence and add its terms to the partial sums (as update_row does).
template <typename XT>
__device__ __forceinline__ void resident_update(double z, double xi, double hi, bool field,
                                                const ResidentArgs& a, XT* xn, int64_t i,
                                                double (&acc)[kNumPartials]) {
    const double y = ddiv(dadd(z, dmul(a.alpha, xi)), a.beta);
    const XT xs = static_cast<XT>(cbrt(y));
    st_coh(xn + i, xs);
    const double d = dsub(static_cast<double>(xs), xi);
    const double x2 = dmul(xi, xi);
    acc[P_X4] = dadd(acc[P_X4], dmul(x2, x2));
    acc[P_X2] = dadd(acc[P_X2], x2);
    acc[P_XZ] = dadd(acc[P_XZ], dmul(xi, z));
    acc[P_DX2] = dadd(acc[P_DX2], dmul(d, d));
    if (field) acc[P_HX] = dadd(acc[P_HX], dmul(hi, xi));
}

// Dense rows: one wavefront per row, the row's couplings in registers
// (JC chunks of 64 columns, n <= 64 JC), x^(k) staged in LDS.
template <typename XT, typename HT, bool FIELD, int JC>
__global__ __launch_bounds__(NT) void resident_dense_kernel(int64_t n, const double* __restrict__ J, int64_t ld,
                                                            const HT* __restrict__ h, ResidentArgs a) {
    __shared__ double xs[64 * JC];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave;
    const bool own = static_cast<int>(blockIdx.x) < a.row_groups && i < n;
    double jr[JC];
#pragma unroll
    for (int u = 0; u < JC; ++u) {
        const int64_t j = lane + u * kWave;
        jr[u] = (own && j < n) ? J[i * ld + j] : 0.0;
    }
    const double hi = (FIELD && own) ? static_cast<double>(h[i]) : 0.0;
    resident_loop<XT, FIELD>(a, n, [&](const XT* xo, XT* xn, double t, double (&acc)[kNumPartials]) {
        // stage x^(k): each thread loads its elements in one batch
        constexpr int PER = (64 * JC + NT - 1) / NT;
        XT v[PER];
#pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int64_t j = threadIdx.x + b * NT;
            v[b] = j < n ? ld_coh(xo + j) : XT(0);
        }
#pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int j = threadIdx.x + b * NT;
            if (j < 64 * JC) xs[j] = static_cast<double>(v[b]);
        }
        __syncthreads();
        if (own) {
            double p = 0.0;
#pragma unroll
            for (int u = 0; u < JC; ++u) {
                const int64_t j = lane + u * kWave;
                if (j < n) p = dadd(p, dmul(jr[u], xs[j]));
            }
            const double z0 = wave_sum(p);
            if (lane == 0) {
                double z = z0;
                if (FIELD) z = dadd(z, dmul(hi, t));
                resident_update<XT>(z, xs[i], hi, FIELD, a, xn, i, acc);
            }
        }
        __syncthreads();
    });
}

// Sparse rows: one lane per row (rows i = w NT + lane, w NT + lane + G NT,
// ...), entries in ascending order, gathers of x^(k) at the point of
// coherence issued eight at a time.  With one row per lane (CACHE > 0) the
// row's first CACHE column indices and values stay in registers for the
// whole run, so an iteration starts with its gathers.
template <typename XT, typename VT>
__device__ __forceinline__ double row_tail(const int32_t* __restrict__ col, const VT* __restrict__ val,
                                           const XT* xo, int e, int e1, double z) {
    for (; e < e1; e += 8) {
        int c[8];
        XT g[8];
        double vv[8];
        // indices past the row's end repeat its last entry, so every load is
        // in bounds and none waits on a branch
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = e + u < e1 ? e + u : e1 - 1;
            c[u] = col[q];
            vv[u] = static_cast<double>(val[q]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) g[u] = ld_coh(xo + c[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e + u < e1) z = dadd(z, dmul(vv[u], static_cast<double>(g[u])));
    }
    return z;
}

template <typename XT, typename VT, typename HT, bool FIELD, int CACHE>
__global__ __launch_bounds__(NT) void resident_csr_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const VT* __restrict__ val,
                                                          const HT* __restrict__ h, ResidentArgs a) {
    const int64_t first = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(a.row_groups) * NT;
    if constexpr (CACHE > 0) {
        // this lane's only row, cached
        const bool own = static_cast<int>(blockIdx.x) < a.row_groups && first < n;
        const int e0 = own ? rp[first] : 0, e1 = own ? rp[first + 1] : 0;
        const int len = e1 - e0;
        int cc[CACHE];
        double cv[CACHE];
#pragma unroll
        for (int u = 0; u < CACHE; ++u) {
            const int q = u < len ? e0 + u : e0;
            cc[u] = u < len ? col[q] : 0;
            cv[u] = u < len ? static_cast<double>(val[q]) : 0.0;
        }
        const double hq = (FIELD && own) ? static_cast<double>(h[first]) : 0.0;
        resident_loop<XT, FIELD>(a, n, [&](const XT* xo, XT* xn, double t, double (&acc)[kNumPartials]) {
            if (!own) return;
            XT g[CACHE];
            const double xi = static_cast<double>(ld_coh(xo + first));
#pragma unroll
            for (int u = 0; u < CACHE; ++u) g[u] = ld_coh(xo + cc[u]);
            double z = 0.0;
#pragma unroll
            for (int u = 0; u < CACHE; ++u)
                if (u < len) z = dadd(z, dmul(cv[u], static_cast<double>(g[u])));
            if (len > CACHE) z = row_tail(col, val, xo, e0 + CACHE, e1, z);
            if (FIELD) z = dadd(z, dmul(hq, t));
            resident_update<XT>(z, xi, hq, FIELD, a, xn, first, acc);
        });
    } else {
        resident_loop<XT, FIELD>(a, n, [&](const XT* xo, XT* xn, double t, double (&acc)[kNumPartials]) {
            for (int64_t i = first; i < n; i += stride) {
                const int e0 = rp[i], e1 = rp[i + 1];
                const double xi = static_cast<double>(ld_coh(xo + i));
                double z = row_tail(col, val, xo, e0, e1, 0.0);
                double hq = 0.0;
                if (FIELD) {
                    hq = static_cast<double>(h[i]);
                    z = dadd(z, dmul(hq, t));
                }
                resident_update<XT>(z, xi, hq, FIELD, a, xn, i, acc);
            }
        });
    }
}

// ---- ADOCH (Alg. 2) resident: stored dense J, no field, one restart ----
//
// Rows as in resident_dense_kernel (a wavefront per row, the row in
// registers, x^(k) staged in LDS from the point of coherence).  The row's
// owner lane keeps x^(k-1)_i and z_{k-1,i} in registers, so of the vectors
// only x^(k) crosses workgroups.  Iteration k:
//   1. z_k,i = (J x^(k))_i; y_i = x_i + c_k (x_i - x^(k-1)_i), (J y)_i =
//      (1 + c_k) z_k,i - c_k z_{k-1,i}; x^(k+1)_i = T(y)_i written before the
//      acceptance test is known; the workgroup's sums of x^4, x^2, x z,
//      y^4, y^2, y (J y), (T(y) - x)^2;
//   2. grid barrier;
//   3. every workgroup adds the G workgroups' sums in the same order,
//      forms H(x^(k)), H(y^(k)), keeps its own copy of the window of the
//      last q + 1 values of H(x) and takes the same decision; workgroup 0
//      logs it;
//   4. y accepted: r^(k) from the sums, Remark S2's test; rejected:
//      x^(k+1)_i = T(x)_i rewritten, its sums, a second barrier, r^(k);
//      H(x^(k)) not finite: x^(k) copied forward and the run ends.
// Every workgroup reaches the same stop at the same iteration, so the loop
// ends without a published stop; barrier waits are bounded as in the DOCH
// run.
template <int NQ>
__device__ void sum_adoch_partials(const double* __restrict__ p, int G, double (&out)[NQ], double* lds) {
#pragma unroll
    for (int j = 0; j < NQ; ++j) out[j] = 0.0;
    for (int g0 = 0; g0 < G; g0 += 4 * NT) {
        double v[4][NQ];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int g = g0 + b * NT + static_cast<int>(threadIdx.x);
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                v[b][j] = g < G ? ld_coh(p + static_cast<size_t>(g) * kAdochResPartials + j) : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int j = 0; j < NQ; ++j) out[j] = dadd(out[j], v[b][j]);
    }
    block_sum<NQ, NT>(out, lds);
}

template <int JC>
__global__ __launch_bounds__(NT) void resident_adoch_dense_kernel(int64_t n, const double* __restrict__ J, int64_t ld,
                                                                  AdochResArgs a) {
    __shared__ double xs[64 * JC];
    __shared__ double red[kAdochResPartials * NW];
    __shared__ double ring[kAdochResMaxW];
    __shared__ int dec[2];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int G = a.row_groups;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave;
    const bool own = i < n;
    const bool owner = own && lane == 0;
    double jr[JC];
#pragma unroll
    for (int u = 0; u < JC; ++u) {
        const int64_t j = lane + u * kWave;
        jr[u] = (own && j < n) ? J[i * ld + j] : 0.0;
    }
    auto xb = [&](int64_t k) { return a.x + (k % 3) * a.xstride; };
    const double b4 = ddiv(a.beta, 4.0), a2 = ddiv(a.alpha, 2.0);
    const int W = a.q + 1;
    double xprev = owner ? ld_coh(xb(0) + i) : 0.0;   // x^(k-1)_i (x^(-1) = x^(0): c_0 = 0)
    double zprev = 0.0;                               // z_{k-1,i}
    unsigned int gen = 0;
    constexpr int PER = (64 * JC + NT - 1) / NT;
    bool staged = false;                // x^(k) already in xs (y accepted last time)
    for (int64_t k = 0; k < a.iters; ++k) {
        const double c = a.cseq[k];
        const double* xo = xb(k);
        double* xn = xb(k + 1);
        double v[PER];
        if (!staged) {
#pragma unroll
            for (int b = 0; b < PER; ++b) {
                const int64_t j = threadIdx.x + b * NT;
                v[b] = j < n ? ld_coh(xo + j) : 0.0;
            }
#pragma unroll
            for (int b = 0; b < PER; ++b) {
                const int j = threadIdx.x + b * NT;
                if (j < 64 * JC) xs[j] = v[b];
            }
            __syncthreads();
        }
        double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double xi = 0.0, zi = 0.0;
        if (own) {
            double p = 0.0;
#pragma unroll
            for (int u = 0; u < JC; ++u) {
                const int64_t j = lane + u * kWave;
                if (j < n) p = dadd(p, dmul(jr[u], xs[j]));
            }
            const double z0 = wave_sum(p);
            if (owner) {
                xi = xs[i];
                zi = z0;
                const double yi = dadd(xi, dmul(c, dsub(xi, xprev)));
                const double jy = dsub(dmul(dadd(1.0, c), zi), dmul(c, zprev));
                const double x2 = dmul(xi, xi), y2 = dmul(yi, yi);
                acc[0] = dmul(x2, x2);
                acc[1] = x2;
                acc[2] = dmul(xi, zi);
                acc[3] = dmul(y2, y2);
                acc[4] = y2;
                acc[5] = dmul(yi, jy);
                const double ty = cbrt(ddiv(dadd(jy, dmul(a.alpha, yi)), a.beta));
                st_coh(xn + i, ty);
                const double d = dsub(ty, xi);
                acc[6] = dmul(d, d);
            }
        }
        block_sum<7, NT>(acc, red);
        double* pk = a.partials + static_cast<size_t>(k & 1) * G * kAdochResPartials;
        if (threadIdx.x == 0)
#pragma unroll
            for (int q = 0; q < 7; ++q) store_agent(pk + static_cast<size_t>(blockIdx.x) * kAdochResPartials + q, acc[q]);
        if (!grid_barrier(a.sync, ++gen, a.state)) return;
        // x^(k+1) = T(y) is requested with the sums: it is the next iterate
        // whenever y is accepted
#pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int64_t j = threadIdx.x + b * NT;
            v[b] = j < n ? ld_coh(xn + j) : 0.0;
        }
        double S[7];
        sum_adoch_partials<7>(pk, G, S, red);
        if (threadIdx.x == 0) {
            const double Hx = dsub(dsub(dmul(b4, S[0]), dmul(a2, S[1])), dmul(0.5, S[2]));
            const double Hy = dsub(dsub(dmul(b4, S[3]), dmul(a2, S[4])), dmul(0.5, S[5]));
            ring[k % W] = Hx;
            const int64_t j0 = k - a.q > 0 ? k - a.q : 0;
            double hmax = Hx;
            for (int64_t j = j0; j <= k; ++j) hmax = fmax(hmax, ring[j % W]);
            const int accept = Hy <= hmax ? 1 : 0;
            int code = isfinite(Hx) ? (accept ? 0 : 1) : 2;
            int stop = code == 2;
            double r = 0.0;
            if (code == 0) {
                r = S[1] == 0.0 ? 0.0 : ddiv(sqrt(S[6]), sqrt(S[1]));
                stop = !isfinite(r) || (a.eps > 0.0 && r < a.eps);
            }
            if (blockIdx.x == 0) {
                RestartState* st = a.state;
                a.log[2 * k] = Hx;
                a.accept_log[k] = static_cast<int8_t>(accept);
                st->H_last = Hx;
                if (code == 2) {
                    st->nonfinite = 1;
                    st->done = 1;
                    st->iters_done = k + 1;
                } else if (code == 0) {
                    a.log[2 * k + 1] = r;
                    st->iters_done = k + 1;
                    st->r_last = r;
                    if (!isfinite(r)) {
                        st->nonfinite = 1;
                        st->done = 1;
                    } else if (a.eps > 0.0 && r < a.eps) {
                        st->converged = 1;
                        st->done = 1;
                    }
                }
            }
            dec[0] = code;
            dec[1] = stop;
        }
        __syncthreads();
        const int code = dec[0];
        int stop = dec[1];
        if (code == 2) {
            if (owner) st_coh(xn + i, xi);
            return;
        }
        if (code == 1) {
            double acc2[2] = {0.0, 0.0};
            if (owner) {
                const double tx = cbrt(ddiv(dadd(zi, dmul(a.alpha, xi)), a.beta));
                st_coh(xn + i, tx);
                const double d = dsub(tx, xi);
                acc2[0] = dmul(d, d);
                acc2[1] = dmul(xi, xi);
            }
            block_sum<2, NT>(acc2, red);
            double* p2 = a.partials + static_cast<size_t>(2) * G * kAdochResPartials;
            if (threadIdx.x == 0)
#pragma unroll
                for (int q = 0; q < 2; ++q) store_agent(p2 + static_cast<size_t>(blockIdx.x) * kAdochResPartials + q, acc2[q]);
            if (!grid_barrier(a.sync, ++gen, a.state)) return;
            double S2[2];
            sum_adoch_partials<2>(p2, G, S2, red);
            if (threadIdx.x == 0) {
                const double r = S2[1] == 0.0 ? 0.0 : ddiv(sqrt(S2[0]), sqrt(S2[1]));
                if (blockIdx.x == 0) {
                    RestartState* st = a.state;
                    a.log[2 * k + 1] = r;
                    st->iters_done = k + 1;
                    st->r_last = r;
                    if (!isfinite(r)) {
                        st->nonfinite = 1;
                        st->done = 1;
                    } else if (a.eps > 0.0 && r < a.eps) {
                        st->converged = 1;
                        st->done = 1;
                    }
                }
                dec[1] = !isfinite(r) || (a.eps > 0.0 && r < a.eps);
            }
            __syncthreads();
            stop = dec[1];
        }
        if (stop) return;
        xprev = xi;
        zprev = zi;
        // every read of xs and dec of this iteration is behind the block
        // sums above; an accepted y leaves x^(k+1) staged for the next one
        staged = code == 0;
        if (staged) {
#pragma unroll
            for (int b = 0; b < PER; ++b) {
                const int j = threadIdx.x + b * NT;
                if (j < 64 * JC) xs[j] = v[b];
            }
        }
        __syncthreads();
    }
}

__global__ void resident_reset_kernel(ResidentSync* sy) {
    unsigned int* w = reinterpret_cast<unsigned int*>(sy);
    for (unsigned int t = threadIdx.x; t < sizeof(ResidentSync) / sizeof(unsigned int); t += blockDim.x) w[t] = 0u;
}

// Cooperative launch of G row workgroups and the reducer; *cap caches how
// many workgroups of this kernel fit on the device at once.
template <typename K>
hipError_t launch_coop(K kern, int* cap, int groups, void** args, hipStream_t s) {
    if (*cap == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, 0);
        if (e != hipSuccess) return e;
        *cap = cus * occ;
    }
    if (groups + 1 > *cap) return hipErrorCooperativeLaunchTooLarge;
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(groups + 1), dim3(NT), args, 0, s);
}

template <typename XT, typename HT, bool FIELD, int JC>
hipError_t launch_dense_t(const DenseView& A, ResidentArgs a, hipStream_t s) {
    static int cap = 0;
    int64_t n = A.n;
    const double* J = A.J;
    int64_t ld = A.ld;
    const HT* h = static_cast<const HT*>(A.h);
    void* args[] = {&n, &J, &ld, &h, &a};
    return launch_coop(resident_dense_kernel<XT, HT, FIELD, JC>, &cap, a.row_groups, args, s);
}

template <typename XT, typename HT, bool FIELD>
hipError_t launch_dense_f(const DenseView& A, const ResidentArgs& a, hipStream_t s) {
    if (A.n <= 1024) return launch_dense_t<XT, HT, FIELD, 16>(A, a, s);
    return launch_dense_t<XT, HT, FIELD, 32>(A, a, s);
}

template <typename XT, typename HT>
hipError_t launch_dense_x(const DenseView& A, const ResidentArgs& a, hipStream_t s) {
    if (A.h) return launch_dense_f<XT, HT, true>(A, a, s);
    return launch_dense_f<XT, HT, false>(A, a, s);
}

template <typename XT, typename VT, typename HT, bool FIELD, int CACHE>
hipError_t launch_csr_t(const CsrView& A, ResidentArgs a, hipStream_t s) {
    static int cap = 0;
    int64_t n = A.n;
    const int32_t* rp = A.rp;
    const int32_t* col = A.col;
    const VT* val = static_cast<const VT*>(A.val);
    const HT* h = static_cast<const HT*>(A.h);
    void* args[] = {&n, &rp, &col, &val, &h, &a};
    return launch_coop(resident_csr_kernel<XT, VT, HT, FIELD, CACHE>, &cap, a.row_groups, args, s);
}

template <typename VT, typename HT, int CACHE>
hipError_t launch_csr_c(const CsrView& A, const ResidentArgs& a, hipStream_t s) {
    if (a.x_dtype == ISING_F64)
        return A.h ? launch_csr_t<double, VT, HT, true, CACHE>(A, a, s) : launch_csr_t<double, VT, HT, false, CACHE>(A, a, s);
    return A.h ? launch_csr_t<float, VT, HT, true, CACHE>(A, a, s) : launch_csr_t<float, VT, HT, false, CACHE>(A, a, s);
}

template <typename VT, typename HT>
hipError_t launch_csr_x(const CsrView& A, const ResidentArgs& a, hipStream_t s) {
    // one row per lane: keep the first 16 entries of each row in registers
    if (A.n <= static_cast<int64_t>(a.row_groups) * NT) return launch_csr_c<VT, HT, 16>(A, a, s);
    return launch_csr_c<VT, HT, 0>(A, a, s);
}

template <int JC>
hipError_t launch_adoch_dense_t(const DenseView& A, AdochResArgs a, hipStream_t s) {
    static int cap = 0;
    int64_t n = A.n;
    const double* J = A.J;
    int64_t ld = A.ld;
    void* args[] = {&n, &J, &ld, &a};
    auto kern = resident_adoch_dense_kernel<JC>;
    if (cap == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, 0);
        if (e != hipSuccess) return e;
        cap = cus * occ;
    }
    if (a.row_groups > cap) return hipErrorCooperativeLaunchTooLarge;
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(a.row_groups), dim3(NT), args, 0, s);
}

}  // namespace

hipError_t launch_resident_adoch_dense(const DenseView& A, const AdochResArgs& a, hipStream_t s) {
    if (A.n > kResidentMaxDense || A.proc_kind != 0 || A.h || a.q + 1 > kAdochResMaxW) return hipErrorInvalidValue;
    if (A.n <= 1024) return launch_adoch_dense_t<16>(A, a, s);
    return launch_adoch_dense_t<32>(A, a, s);
}

int resident_row_groups(bool dense, int64_t n) {
    if (dense) return static_cast<int>((n + NW - 1) / NW);
    const int64_t g = (n + NT - 1) / NT;
    return static_cast<int>(g < kResidentMaxCsrGroups ? g : kResidentMaxCsrGroups);
}

hipError_t launch_resident_reset(ResidentSync* sy, hipStream_t s) {
    hipLaunchKernelGGL(resident_reset_kernel, dim3(1), dim3(256), 0, s, sy);
    return hipGetLastError();
}

hipError_t launch_resident_dense(const DenseView& A, const ResidentArgs& a, hipStream_t s) {
    if (A.n > kResidentMaxDense || A.proc_kind != 0) return hipErrorInvalidValue;
    const bool h64 = A.h && A.ht == ISING_F64;
    if (a.x_dtype == ISING_F64) return h64 ? launch_dense_x<double, double>(A, a, s) : launch_dense_x<double, float>(A, a, s);
    return h64 ? launch_dense_x<float, double>(A, a, s) : launch_dense_x<float, float>(A, a, s);
}

hipError_t launch_resident_csr(const CsrView& A, const ResidentArgs& a, hipStream_t s) {
    const bool h64 = A.h && A.ht == ISING_F64;
    if (A.vt == ISING_I16) return h64 ? launch_csr_x<int16_t, double>(A, a, s) : launch_csr_x<int16_t, float>(A, a, s);
    if (A.vt == ISING_F64) return h64 ? launch_csr_x<double, double>(A, a, s) : launch_csr_x<double, float>(A, a, s);
    return h64 ? launch_csr_x<float, double>(A, a, s) : launch_csr_x<float, float>(A, a, s);
}

}  // namespace doch
