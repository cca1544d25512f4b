// kernels_csr.hip -- sparse (CSR) kernels of the DOCH hot path for gfx950.
//
// One DOCH iteration (Methods, eq:FPE / Alg. 1) on a CSR coupling matrix is a
// single streaming pass: row blocks of up to 256 rows and 2048 stored
// entries are assigned to workgroups; a workgroup streams the block's column
// indices and values with non-temporal loads (they are used once per
// iteration, so they should not evict the iterate from L2), gathers the
// iterate, parks the products in LDS, and then one thread per row sums its
// products in ascending column order, applies the cube-root update and adds
// to the iteration's FP64 partial sums.  The last workgroup finishes the
// iteration (H, r, the field spin) -- see step_common.h.
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

template <typename XT, typename VT, typename HT, bool FIELD>
__global__ __launch_bounds__(NT) void csr_step_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h,
    const int32_t* __restrict__ blk, int64_t nblk, StepArgs a) {
    if (a.state->done) return;
    __shared__ double prod[kBlockNnz];
    __shared__ double red[kNumPartials * NW];
    const XT* __restrict__ x = static_cast<const XT*>(a.x_old);
    XT* __restrict__ xn = static_cast<XT*>(a.x_new);
    const double t_old = FIELD ? static_cast<double>(x[n]) : 0.0;
    double acc[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;

    int64_t b, bend, bstep;
    block_range(nblk, b, bend, bstep);
    for (; b < bend; b += bstep) {
        const int r0 = blk[b], r1 = blk[b + 1];
        const int e0 = rp[r0], e1 = rp[r1];
        const int cnt = e1 - e0;
        if (cnt <= kBlockNnz) {
            for (int e = threadIdx.x; e < cnt; e += NT) {
                const int c = ld_stream(col + e0 + e);
                const double v = static_cast<double>(ld_stream(val + e0 + e));
                prod[e] = dmul(v, static_cast<double>(x[c]));
            }
            __syncthreads();
            const int i = r0 + static_cast<int>(threadIdx.x);
            if (i < r1) {
                const int lo = rp[i] - e0, hi = rp[i + 1] - e0;
                double z = 0.0;
                for (int e = lo; e < hi; ++e) z = dadd(z, prod[e]);
                double hv = 0.0;
                if (FIELD) {
                    hv = static_cast<double>(ld_stream(h + i));
                    z = dadd(z, dmul(hv, t_old));
                }
                update_row<XT>(z, static_cast<double>(x[i]), hv, FIELD, a, xn, i, acc);
            }
            __syncthreads();
        } else {
            // one long row: the whole workgroup reduces it
            double part[1] = {0.0};
            for (int e = threadIdx.x; e < cnt; e += NT) {
                const int c = ld_stream(col + e0 + e);
                const double v = static_cast<double>(ld_stream(val + e0 + e));
                part[0] = dadd(part[0], dmul(v, static_cast<double>(x[c])));
            }
            block_sum<1, NT>(part, red);
            if (threadIdx.x == 0) {
                double z = part[0];
                double hv = 0.0;
                if (FIELD) {
                    hv = static_cast<double>(h[r0]);
                    z = dadd(z, dmul(hv, t_old));
                }
                update_row<XT>(z, static_cast<double>(x[r0]), hv, FIELD, a, xn, r0, acc);
            }
            __syncthreads();
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

// ------------------------------------------------------------ validation
// flags[0]: malformed CSR, flags[1]: nonzero diagonal, flags[2]: a value is
// not an integer of magnitude < 2^31.
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
        last_flag = arrive_last(ticket, gridDim.x) ? 1 : 0;
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
        last_flag = arrive_last(ticket, gridDim.x) ? 1 : 0;
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

int csr_step_grid(int64_t nblk) {
    if (nblk < 64) return static_cast<int>(nblk < 1 ? 1 : nblk);
    int64_t g = nblk < 2048 ? nblk : 2048;
    return static_cast<int>(g & ~static_cast<int64_t>(7));
}

#define DOCH_DISPATCH_VT_HT(A, BODY)                                              \
    do {                                                                          \
        if ((A).vt == ISING_F64 && (A).ht == ISING_F64) {                         \
            using VT = double; using HT = double; BODY;                           \
        } else if ((A).vt == ISING_F64) {                                         \
            using VT = double; using HT = float; BODY;                            \
        } else if ((A).ht == ISING_F64) {                                         \
            using VT = float; using HT = double; BODY;                            \
        } else {                                                                  \
            using VT = float; using HT = float; BODY;                             \
        }                                                                         \
    } while (0)

hipError_t launch_csr_step(const CsrView& A, const int32_t* blk, int64_t nblk,
                           const StepArgs& a, int grid, hipStream_t s) {
    const bool field = A.h != nullptr;
    DOCH_DISPATCH_VT_HT(A, {
        const VT* val = static_cast<const VT*>(A.val);
        const HT* h = static_cast<const HT*>(A.h);
        if (a.x_dtype == ISING_F64) {
            if (field)
                hipLaunchKernelGGL((csr_step_kernel<double, VT, HT, true>), dim3(grid), dim3(NT), 0, s,
                                   A.n, A.rp, A.col, val, h, blk, nblk, a);
            else
                hipLaunchKernelGGL((csr_step_kernel<double, VT, HT, false>), dim3(grid), dim3(NT), 0, s,
                                   A.n, A.rp, A.col, val, h, blk, nblk, a);
        } else {
            if (field)
                hipLaunchKernelGGL((csr_step_kernel<float, VT, HT, true>), dim3(grid), dim3(NT), 0, s,
                                   A.n, A.rp, A.col, val, h, blk, nblk, a);
            else
                hipLaunchKernelGGL((csr_step_kernel<float, VT, HT, false>), dim3(grid), dim3(NT), 0, s,
                                   A.n, A.rp, A.col, val, h, blk, nblk, a);
        }
    });
    return hipGetLastError();
}

hipError_t launch_csr_energy(const CsrView& A, const int8_t* s_spins, int R,
                             double* partials, unsigned int* ticket, int grid,
                             double* E, int64_t* E_int, hipStream_t s) {
    const bool field = A.h != nullptr;
    const int want_int = E_int != nullptr;
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
    else
        hipLaunchKernelGGL(csr_validate_kernel<float>, dim3(grid), dim3(NT), 0, s, A.n, A.nnz,
                           A.rp, A.col, static_cast<const float*>(A.val), flags);
    return hipGetLastError();
}

hipError_t launch_csr_symcheck(const CsrView& A, int32_t* bad, hipStream_t s) {
    const int grid = grid_for_rows(A.n);
    if (A.vt == ISING_F64)
        hipLaunchKernelGGL(csr_symcheck_kernel<double>, dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, static_cast<const double*>(A.val), bad);
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
