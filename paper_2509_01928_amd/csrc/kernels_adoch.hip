// kernels_adoch.hip -- accelerated DOCH (Alg. 2, eq:BBscheme) on CSR, and
// the update and output steps it shares with the dense matvec.
//
// Iteration k needs H(x^(k)), H(y^(k)) with y = x^(k) + c_k (x^(k) - x^(k-1)),
// c_k = (t_k - 1) / t_{k+1}, and then x^(k+1) = T(v), v = y or x^(k).  All of
// it costs one matvec: with z_k = Jhat x^(k) kept from this iteration and
// z_{k-1} from the last, Jhat y = (1 + c_k) z_k - c_k z_{k-1} and Jhat v is
// one of the two.  Two launches per iteration:
//   adoch_mv_kernel     z_k, the partial sums of H(x^(k)) and H(y^(k)); its
//                       last workgroup finishes both, keeps the window of
//                       the last q+1 values of H(x) and decides whether y is
//                       accepted (H(y) <= max of the window), per restart;
//                       on CSR it also writes x^(k+1) = T(y^(k)) before that
//                       decision is known, with the sums of r^(k), and
//                       closes every restart whose y is accepted;
//   adoch_update_kernel x^(k+1) = cbrt((Jhat v + alpha v) / beta) elementwise
//                       (the extra field spin included) and r^(k): after
//                       the dense product for every restart, after the CSR
//                       one only for those whose y was rejected.
// R restarts (1, 2, 4 or 8) run together, interleaved (entry (i, r) at
// i R + r), each with its own window, decisions and stopping; a stopped
// restart is copied forward unchanged.  Iterates rotate through three
// buffers (x^(k-1), x^(k), x^(k+1)), products through two.  FP64 throughout.
#include "adoch_common.h"

#include <type_traits>
#include "device_common.h"
#include "ising_internal.h"

namespace doch {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;

// RL = 4: every row holds 4 entries starting at 4 i (the lattice), read as
// one 16-byte chunk of indices and one of values without the row offsets;
// RL = 0: offsets read, entries one at a time.  Same order either way.
//
// OPT: the product also writes x^(k+1) = T(y^(k)) = cbrt((Jhat y + alpha y)
// / beta) of every restart that has not stopped (a stopped one is copied
// forward), optimistically, before the acceptance test that follows the
// global sums, and adds |T(y) - x^(k)|^2 as an eighth sum.  y is taken far
// more often than not, and then x^(k+1) and r^(k) are final when the launch
// ends: the second pass over x^(k), x^(k-1), z_k, z_(k-1) and x^(k+1) is
// made only for a rejected restart (adoch_update_kernel's fix-up mode).
// The value written is the one the update would write, bit for bit.
// CT: int32_t = column indices; int16_t (4-entry rows only) = each entry's
// cyclic column offset col - i, taken into [-32768, 32767] modulo n.
template <typename VT, typename HT, bool FIELD, int RL, int R, bool OPT, typename CT = int32_t>
__global__ __launch_bounds__(NT) void adoch_mv_kernel(
    int64_t n, const int32_t* __restrict__ rp, const CT* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, const double* __restrict__ x,
    const double* __restrict__ xp, const double* __restrict__ zp, double* __restrict__ z,
    double* __restrict__ xn, AdochArgs a) {
    if (*a.all_done) return;
    constexpr int S = OPT ? 8 : 7;
    __shared__ double red[S * R * NW];
    __shared__ int last_flag;
    const double c = a.c;
    const double al = a.alpha, be = a.beta;
    double tx[R];
    bool live[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        tx[r] = FIELD ? x[n * R + r] : 0.0;
        live[r] = OPT ? a.state[r].done == 0 : true;
    }
    // per restart: x^4, x^2, x z, y^4, y^2, y (Jy), h x [, |T(y) - x|^2]
    double acc[S * R];
#pragma unroll
    for (int q = 0; q < S * R; ++q) acc[q] = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        double zi[R];
#pragma unroll
        for (int r = 0; r < R; ++r) zi[r] = 0.0;
        if constexpr (RL == 4) {
            const auto cv = ld_stream4(col + 4 * i);
            const auto vv = ld_stream4(val + 4 * i);
            int64_t cc[4] = {cv.x, cv.y, cv.z, cv.w};
            if constexpr (sizeof(CT) == 2) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    cc[q] += i;
                    cc[q] += cc[q] < 0 ? n : 0;
                    cc[q] -= cc[q] >= n ? n : 0;
                }
            }
            const double v[4] = {static_cast<double>(vv.x), static_cast<double>(vv.y),
                                 static_cast<double>(vv.z), static_cast<double>(vv.w)};
            double g[4][R];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) g[q][r] = x[cc[q] * R + r];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) zi[r] = dadd(zi[r], dmul(v[q], g[q][r]));
        } else {
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const double v = static_cast<double>(val[e]);
                const int64_t j = col[e];
#pragma unroll
                for (int r = 0; r < R; ++r) zi[r] = dadd(zi[r], dmul(v, x[j * R + r]));
            }
        }
        const double hi = FIELD ? static_cast<double>(h[i]) : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t t = i * R + r;
            const double xi = x[t];
            double zr = zi[r];
            if (FIELD) {
                zr = dadd(zr, dmul(hi, tx[r]));
                acc[S * r + 6] = dadd(acc[S * r + 6], dmul(hi, xi));
            }
            // x^(k-1), z_(k-1) and z_k are streamed (read or written once
            // per iteration); x^(k) is also gathered by other rows and stays
            // cached
            if constexpr (OPT) __builtin_nontemporal_store(zr, z + t);
            else z[t] = zr;
            const double xpt = OPT ? ld_stream(xp + t) : xp[t];
            const double zpt = OPT ? ld_stream(zp + t) : zp[t];
            const double yi = dadd(xi, dmul(c, dsub(xi, xpt)));
            const double jy = dsub(dmul(dadd(1.0, c), zr), dmul(c, zpt));
            const double x2 = dmul(xi, xi), y2 = dmul(yi, yi);
            acc[S * r + 0] = dadd(acc[S * r + 0], dmul(x2, x2));
            acc[S * r + 1] = dadd(acc[S * r + 1], x2);
            acc[S * r + 2] = dadd(acc[S * r + 2], dmul(xi, zr));
            acc[S * r + 3] = dadd(acc[S * r + 3], dmul(y2, y2));
            acc[S * r + 4] = dadd(acc[S * r + 4], y2);
            acc[S * r + 5] = dadd(acc[S * r + 5], dmul(yi, jy));
            if constexpr (OPT) {
                double nx = xi;
                if (live[r]) {
                    nx = cbrt(ddiv(dadd(jy, dmul(al, yi)), be));
                    const double d = dsub(nx, xi);
                    acc[S * r + 7] = dadd(acc[S * r + 7], dmul(d, d));
                }
                __builtin_nontemporal_store(nx, xn + t);
            }
        }
    }
    block_sum<S * R, NT>(acc, red);
    adoch_mv_close<R, NT, FIELD, OPT>(acc, red, &last_flag, n, x, xp, zp, z, a, xn);
}

// x^(k+1) of every restart that has not stopped (a stopped one is copied
// forward), and r^(k) = |x^(k+1) - x^(k)| / |x^(k)| per restart; the last
// workgroup applies Remark S2's test and raises all_done when every restart
// has stopped.
//
// FIXUP (after the optimistic CSR product): only the restarts the product's
// closing step marked are touched: fix = 1 (y rejected) gets x^(k+1) =
// T(x^(k)) and its r^(k) and stopping test here, fix = 2 (H(x^(k)) not
// finite) has x^(k) copied forward; the launch returns at once when nothing
// is marked, and its last workgroup clears the marks.
template <int R, bool FIXUP>
__global__ __launch_bounds__(NT) void adoch_update_kernel(
    int64_t np, const double* __restrict__ x, const double* __restrict__ xp,
    const double* __restrict__ z, const double* __restrict__ zp, double* __restrict__ xn,
    AdochArgs a) {
    if (*a.all_done) return;
    if (FIXUP && !a.fix[8]) return;
    __shared__ double red[2 * R * NW];
    __shared__ int last_flag;
    const double c = a.c;
    // a thread's entries t = i R + r all have the same restart r (the grid
    // stride is a multiple of R)
    const int myr = static_cast<int>((static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x) % R);
    const int code = FIXUP ? a.fix[myr] : 0;
    const bool stopped = FIXUP ? code == 2 : a.state[myr].done != 0;
    const bool acc_y = FIXUP ? false : a.accept[myr] != 0;
    const bool idle = FIXUP && code == 0;
    double d2 = 0.0, x2 = 0.0;        // (x^(k+1) - x^(k))^2, x^(k)^2
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < np * R && !idle;
         t += static_cast<int64_t>(gridDim.x) * NT) {
        const double xi = x[t];
        if (stopped) {
            xn[t] = xi;
            continue;
        }
        double v = xi, jv = z[t];
        if (acc_y) {
            v = dadd(xi, dmul(c, dsub(xi, xp[t])));
            jv = dsub(dmul(dadd(1.0, c), z[t]), dmul(c, zp[t]));
        }
        const double nx = cbrt(ddiv(dadd(jv, dmul(a.alpha, v)), a.beta));
        xn[t] = nx;
        const double d = dsub(nx, xi);
        d2 = dadd(d2, dmul(d, d));
        x2 = dadd(x2, dmul(xi, xi));
    }
    double acc[2 * R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[2 * r] = r == myr ? d2 : 0.0;
        acc[2 * r + 1] = r == myr ? x2 : 0.0;
    }
    block_sum<2 * R, NT>(acc, red);
    if (threadIdx.x == 0) {
        double* p = a.partials + static_cast<size_t>(blockIdx.x) * 2 * R;
#pragma unroll
        for (int q = 0; q < 2 * R; ++q) store_agent(p + q, acc[q]);
        last_flag = arrive_last_grid(a.ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[2 * R];
#pragma unroll
    for (int q = 0; q < 2 * R; ++q) u[q] = 0.0;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT)
#pragma unroll
        for (int q = 0; q < 2 * R; ++q) u[q] = dadd(u[q], load_agent(a.partials + static_cast<size_t>(g) * 2 * R + q));
    block_sum<2 * R, NT>(u, red);
    // one thread per restart (each closing is a chain of global accesses)
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 2 * R; ++q) red[q] = u[q];
    __syncthreads();
    __shared__ int rdone[R];
    const int r = threadIdx.x;
    if (r < R) {
        RestartState* st = a.state + r;
        const bool mine = FIXUP ? a.fix[r] == 1 : !st->done;
        if (FIXUP) a.fix[r] = 0;
        if (mine) {
            const double d2 = red[2 * r], x2 = red[2 * r + 1];
            const double rr = x2 == 0.0 ? 0.0 : ddiv(sqrt(d2), sqrt(x2));
            a.log[(static_cast<size_t>(a.k) * R + r) * 2 + 1] = rr;
            st->iters_done = a.k + 1;
            st->r_last = rr;
            if (!isfinite(rr)) {
                st->nonfinite = 1;
                st->done = 1;
            } else if (a.eps > 0.0 && rr < a.eps) {
                st->converged = 1;
                st->done = 1;
            }
        }
        rdone[r] = st->done;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int all = 1;
    for (int q = 0; q < R; ++q) all &= rdone[q];
    if (FIXUP) a.fix[8] = 0;
    if (all) *a.all_done = 1;
    reset_ticket(a.ticket);
}

// Every restart's last iterate sits in buffer K mod 3, K = the largest
// iters_done (stopped restarts were copied forward until the last one
// stopped).
__global__ __launch_bounds__(NT) void adoch_finish_kernel(const double* __restrict__ b0,
                                                          const double* __restrict__ b1,
                                                          const double* __restrict__ b2,
                                                          const RestartState* __restrict__ st,
                                                          int64_t n, int64_t np, int R, int field,
                                                          double* __restrict__ x_out,
                                                          int8_t* __restrict__ s_out) {
    int64_t kmax = 0;
    for (int r = 0; r < R; ++r) kmax = st[r].iters_done > kmax ? st[r].iters_done : kmax;
    const int64_t m = kmax % 3;
    const double* xb = m == 0 ? b0 : (m == 1 ? b1 : b2);
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < np * R;
         t += static_cast<int64_t>(gridDim.x) * NT) {
        const double v = xb[t];
        if (x_out) x_out[t] = v;
        const int64_t i = t / R;
        if (s_out && i < n) {
            int s = v >= 0.0 ? 1 : -1;
            if (field && !(xb[n * R + t % R] >= 0.0)) s = -s;
            s_out[t] = static_cast<int8_t>(s);
        }
    }
}

int grid_rows(int64_t n) {
    int64_t g = (n + NT - 1) / NT;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

int adoch_grid(int64_t n) { return grid_rows(n); }

#define DOCH_ADOCH_R(R, ...)                               \
    switch (R) {                                           \
        case 1: { constexpr int RR = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int RR = 2; __VA_ARGS__; } break; \
        case 4: { constexpr int RR = 4; __VA_ARGS__; } break; \
        case 8: { constexpr int RR = 8; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;              \
    }

template <typename VT, typename HT, bool F, int RR>
static void adoch_mv_go(const CsrView& A, int grid, const double* x, const double* xp, const double* zp,
                        double* z, double* xn, const AdochArgs& a, hipStream_t s) {
    const VT* v = static_cast<const VT*>(A.val);
    const HT* h = static_cast<const HT*>(A.h);
    if constexpr (std::is_same<VT, int8_t>::value) {
        // 4-entry rows with the 16-bit column offsets (kept with the 8-bit values)
        if (A.col16 && A.row_len == 4) {
            if (xn)
                hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 4, RR, true, int16_t>), dim3(grid), dim3(NT), 0, s,
                                   A.n, A.rp, A.col16, v, h, x, xp, zp, z, xn, a);
            else
                hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 4, RR, false, int16_t>), dim3(grid), dim3(NT), 0, s,
                                   A.n, A.rp, A.col16, v, h, x, xp, zp, z, xn, a);
            return;
        }
    }
    if (A.row_len == 4 && xn)
        hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 4, RR, true>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, x, xp, zp, z, xn, a);
    else if (A.row_len == 4)
        hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 4, RR, false>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, x, xp, zp, z, xn, a);
    else if (xn)
        hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 0, RR, true>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, x, xp, zp, z, xn, a);
    else
        hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 0, RR, false>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, x, xp, zp, z, xn, a);
}

template <typename VT, int RR>
static void adoch_mv_vt(const CsrView& A, int grid, const double* x, const double* xp, const double* zp,
                        double* z, double* xn, const AdochArgs& a, hipStream_t s) {
    if (!A.h) adoch_mv_go<VT, float, false, RR>(A, grid, x, xp, zp, z, xn, a, s);
    else if (A.ht == ISING_F64) adoch_mv_go<VT, double, true, RR>(A, grid, x, xp, zp, z, xn, a, s);
    else adoch_mv_go<VT, float, true, RR>(A, grid, x, xp, zp, z, xn, a, s);
}

hipError_t launch_adoch_mv(const CsrView& A, const double* x, const double* xp, const double* zp,
                           double* z, double* xn, const AdochArgs& a, hipStream_t s) {
    int grid = grid_rows(A.n);
    // small-integer couplings on 4-entry rows: the library's exact 8-bit
    // copy of the values is streamed instead (a quarter of the FP32 bytes)
    const bool i8 = A.val8 && A.row_len == 4;
    if (A.row_len == 4) {
        // rows of 4 entries with implicit offsets stream best with few
        // workgroups per compute unit, each lane walking many rows
        // (measured on the 10^8-spin lattice, one restart; FP32 values:
        // 1395 us per iteration with 2 per CU against 1789 with 8, 1522
        // with 4, 1658 with 1.5 and 1947 with 1; 8-bit values: 1201 us with
        // 3 against 1275 with 2 and 1237 with 4; 8-bit values and 16-bit
        // column offsets: 1101 us with 4 against 1117 with 3, 1203 with 6
        // and 1399 with 8)
        const int wpc = i8 ? (A.col16 ? 4 : 3) : 2;
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0 &&
            grid > wpc * cus)
            grid = wpc * cus;
    }
    CsrView B = A;
    if (i8) B.val = A.val8;
    DOCH_ADOCH_R(a.R, {
        if (i8) adoch_mv_vt<int8_t, RR>(B, grid, x, xp, zp, z, xn, a, s);
        else if (A.vt == ISING_I16) adoch_mv_vt<int16_t, RR>(A, grid, x, xp, zp, z, xn, a, s);
        else if (A.vt == ISING_F64) adoch_mv_vt<double, RR>(A, grid, x, xp, zp, z, xn, a, s);
        else adoch_mv_vt<float, RR>(A, grid, x, xp, zp, z, xn, a, s);
    });
    return hipGetLastError();
}

hipError_t launch_adoch_update(int64_t np, const double* x, const double* xp, const double* z,
                               const double* zp, double* xn, const AdochArgs& a, bool fixup, hipStream_t s) {
    const int grid = grid_rows(np * a.R);
    DOCH_ADOCH_R(a.R, {
        if (fixup)
            hipLaunchKernelGGL((adoch_update_kernel<RR, true>), dim3(grid), dim3(NT), 0, s, np, x, xp, z, zp, xn, a);
        else
            hipLaunchKernelGGL((adoch_update_kernel<RR, false>), dim3(grid), dim3(NT), 0, s, np, x, xp, z, zp, xn,
                               a);
    });
    return hipGetLastError();
}

hipError_t launch_adoch_finish(const double* b0, const double* b1, const double* b2,
                               const RestartState* st, int64_t n, int64_t np, int R, bool field,
                               double* x_out, int8_t* s_out, hipStream_t s) {
    hipLaunchKernelGGL(adoch_finish_kernel, dim3(grid_rows(np * R)), dim3(NT), 0, s, b0, b1, b2, st, n, np, R,
                       field ? 1 : 0, x_out, s_out);
    return hipGetLastError();
}

}  // namespace doch
