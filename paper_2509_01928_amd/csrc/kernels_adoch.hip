// kernels_adoch.hip -- accelerated DOCH (Alg. 2, eq:BBscheme) on CSR.
//
// Iteration k needs H(x^(k)), H(y^(k)) with y = x^(k) + c_k (x^(k) - x^(k-1)),
// c_k = (t_k - 1) / t_{k+1}, and then x^(k+1) = T(v), v = y or x^(k).  All of
// it costs one matvec: with z_k = Jhat x^(k) kept from this iteration and
// z_{k-1} from the last, Jhat y = (1 + c_k) z_k - c_k z_{k-1} and Jhat v is
// one of the two.  Two launches per iteration:
//   adoch_mv_kernel     z_k, the partial sums of H(x^(k)) and H(y^(k)); its
//                       last workgroup finishes both, keeps the window of
//                       the last q+1 values of H(x) and decides whether y is
//                       accepted (H(y) <= max of the window);
//   adoch_update_kernel x^(k+1) = cbrt((Jhat v + alpha v) / beta) elementwise
//                       (the extra field spin included) and r^(k).
// Iterates rotate through three buffers (x^(k-1), x^(k), x^(k+1)), products
// through two.  FP64 throughout.
#include "device_common.h"
#include "ising_internal.h"

namespace doch {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;

// RL = 4: every row holds 4 entries starting at 4 i (the lattice), read as
// one 16-byte chunk of indices and one of values without the row offsets;
// RL = 0: offsets read, entries one at a time.  Same order either way.
template <typename VT, typename HT, bool FIELD, int RL>
__global__ __launch_bounds__(NT) void adoch_mv_kernel(
    int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const VT* __restrict__ val, const HT* __restrict__ h, const double* __restrict__ x,
    const double* __restrict__ xp, const double* __restrict__ zp, double* __restrict__ z,
    AdochArgs a) {
    if (a.state->done) return;
    __shared__ double red[7 * NW];
    __shared__ int last_flag;
    const double c = a.c;
    const double tx = FIELD ? x[n] : 0.0;
    // x^4, x^2, x z, y^4, y^2, y (Jy), h x
    double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        double zi = 0.0;
        if constexpr (RL == 4) {
            const auto cv = ld_stream4(col + 4 * i);
            const auto vv = ld_stream4(val + 4 * i);
            const double g[4] = {x[cv.x], x[cv.y], x[cv.z], x[cv.w]};
            const double v[4] = {static_cast<double>(vv.x), static_cast<double>(vv.y),
                                 static_cast<double>(vv.z), static_cast<double>(vv.w)};
#pragma unroll
            for (int q = 0; q < 4; ++q) zi = dadd(zi, dmul(v[q], g[q]));
        } else {
            for (int e = rp[i]; e < rp[i + 1]; ++e) zi = dadd(zi, dmul(static_cast<double>(val[e]), x[col[e]]));
        }
        const double xi = x[i];
        if (FIELD) {
            const double hi = static_cast<double>(h[i]);
            zi = dadd(zi, dmul(hi, tx));
            acc[6] = dadd(acc[6], dmul(hi, xi));
        }
        z[i] = zi;
        const double yi = dadd(xi, dmul(c, dsub(xi, xp[i])));
        const double jy = dsub(dmul(dadd(1.0, c), zi), dmul(c, zp[i]));
        const double x2 = dmul(xi, xi), y2 = dmul(yi, yi);
        acc[0] = dadd(acc[0], dmul(x2, x2));
        acc[1] = dadd(acc[1], x2);
        acc[2] = dadd(acc[2], dmul(xi, zi));
        acc[3] = dadd(acc[3], dmul(y2, y2));
        acc[4] = dadd(acc[4], y2);
        acc[5] = dadd(acc[5], dmul(yi, jy));
    }
    block_sum<7, NT>(acc, red);
    if (threadIdx.x == 0) {
        double* p = a.partials + static_cast<size_t>(blockIdx.x) * 7;
        for (int q = 0; q < 7; ++q) store_agent(p + q, acc[q]);
        last_flag = arrive_last_grid(a.ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT)
        for (int q = 0; q < 7; ++q) u[q] = dadd(u[q], load_agent(a.partials + g * 7 + q));
    block_sum<7, NT>(u, red);
    if (threadIdx.x != 0) return;
    if (FIELD) {
        // the extra spin's row: z_n = sum_i h_i x_i, and its share of every sum
        const double zn = u[6];
        z[n] = zn;
        const double yn = dadd(tx, dmul(c, dsub(tx, xp[n])));
        const double jyn = dsub(dmul(dadd(1.0, c), zn), dmul(c, zp[n]));
        const double t2 = dmul(tx, tx), y2 = dmul(yn, yn);
        u[0] = dadd(u[0], dmul(t2, t2));
        u[1] = dadd(u[1], t2);
        u[2] = dadd(u[2], dmul(tx, zn));
        u[3] = dadd(u[3], dmul(y2, y2));
        u[4] = dadd(u[4], y2);
        u[5] = dadd(u[5], dmul(yn, jyn));
    }
    const double b4 = ddiv(a.beta, 4.0), a2 = ddiv(a.alpha, 2.0);
    const double Hx = dsub(dsub(dmul(b4, u[0]), dmul(a2, u[1])), dmul(0.5, u[2]));
    const double Hy = dsub(dsub(dmul(b4, u[3]), dmul(a2, u[4])), dmul(0.5, u[5]));
    // window of H(x^(j)), max(0, k - q) <= j <= k
    a.ring[a.k % (a.q + 1)] = Hx;
    const int64_t j0 = a.k - a.q > 0 ? a.k - a.q : 0;
    double hmax = Hx;
    for (int64_t j = j0; j <= a.k; ++j) hmax = fmax(hmax, a.ring[j % (a.q + 1)]);
    const int accept = Hy <= hmax ? 1 : 0;
    *a.accept = accept;
    a.log[2 * a.k] = Hx;
    a.accept_log[a.k] = static_cast<int8_t>(accept);
    a.state->H_last = Hx;
    if (!isfinite(Hx)) {
        a.state->nonfinite = 1;
        a.state->done = 1;
        a.state->iters_done = a.k + 1;
    }
    reset_ticket(a.ticket);
}

__global__ __launch_bounds__(NT) void adoch_update_kernel(
    int64_t np, const double* __restrict__ x, const double* __restrict__ xp,
    const double* __restrict__ z, const double* __restrict__ zp, double* __restrict__ xn,
    AdochArgs a) {
    if (a.state->done) return;
    __shared__ double red[2 * NW];
    __shared__ int last_flag;
    const double c = a.c;
    const bool acc_y = *a.accept != 0;
    double acc[2] = {0.0, 0.0};        // (x^(k+1) - x^(k))^2, x^(k)^2
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < np;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        const double xi = x[i];
        double v = xi, jv = z[i];
        if (acc_y) {
            v = dadd(xi, dmul(c, dsub(xi, xp[i])));
            jv = dsub(dmul(dadd(1.0, c), z[i]), dmul(c, zp[i]));
        }
        const double nx = cbrt(ddiv(dadd(jv, dmul(a.alpha, v)), a.beta));
        xn[i] = nx;
        const double d = dsub(nx, xi);
        acc[0] = dadd(acc[0], dmul(d, d));
        acc[1] = dadd(acc[1], dmul(xi, xi));
    }
    block_sum<2, NT>(acc, red);
    if (threadIdx.x == 0) {
        double* p = a.partials + static_cast<size_t>(blockIdx.x) * 2;
        store_agent(p, acc[0]);
        store_agent(p + 1, acc[1]);
        last_flag = arrive_last_grid(a.ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[2] = {0.0, 0.0};
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT) {
        u[0] = dadd(u[0], load_agent(a.partials + g * 2));
        u[1] = dadd(u[1], load_agent(a.partials + g * 2 + 1));
    }
    block_sum<2, NT>(u, red);
    if (threadIdx.x != 0) return;
    const double r = u[1] == 0.0 ? 0.0 : ddiv(sqrt(u[0]), sqrt(u[1]));
    a.log[2 * a.k + 1] = r;
    RestartState* st = a.state;
    st->iters_done = a.k + 1;
    st->r_last = r;
    if (!isfinite(r)) {
        st->nonfinite = 1;
        st->done = 1;
    } else if (a.eps > 0.0 && r < a.eps) {
        st->converged = 1;
        st->done = 1;
    }
    reset_ticket(a.ticket);
}

// x^(iters_done) sits in buffer iters_done mod 3.
__global__ __launch_bounds__(NT) void adoch_finish_kernel(const double* __restrict__ b0,
                                                          const double* __restrict__ b1,
                                                          const double* __restrict__ b2,
                                                          const RestartState* __restrict__ st,
                                                          int64_t n, int64_t np, int field,
                                                          double* __restrict__ x_out,
                                                          int8_t* __restrict__ s_out) {
    const int64_t m = st->iters_done % 3;
    const double* xb = m == 0 ? b0 : (m == 1 ? b1 : b2);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < np;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        const double v = xb[i];
        if (x_out) x_out[i] = v;
        if (s_out && i < n) {
            int s = v >= 0.0 ? 1 : -1;
            if (field && !(xb[n] >= 0.0)) s = -s;
            s_out[i] = static_cast<int8_t>(s);
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

hipError_t launch_adoch_mv(const CsrView& A, const double* x, const double* xp, const double* zp,
                           double* z, const AdochArgs& a, hipStream_t s) {
    const int grid = grid_rows(A.n);
    const bool field = A.h != nullptr;
#define DOCH_ADOCH_MV(VT, HT, F)                                                                   \
    do {                                                                                           \
        if (A.row_len == 4)                                                                        \
            hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 4>), dim3(grid), dim3(NT), 0, s, A.n, A.rp, \
                               A.col, static_cast<const VT*>(A.val), static_cast<const HT*>(A.h), x, xp, \
                               zp, z, a);                                                          \
        else                                                                                       \
            hipLaunchKernelGGL((adoch_mv_kernel<VT, HT, F, 0>), dim3(grid), dim3(NT), 0, s, A.n, A.rp, \
                               A.col, static_cast<const VT*>(A.val), static_cast<const HT*>(A.h), x, xp, \
                               zp, z, a);                                                          \
    } while (0)
    if (A.vt == ISING_I16) {
        if (!field) DOCH_ADOCH_MV(int16_t, float, false);
        else if (A.ht == ISING_F64) DOCH_ADOCH_MV(int16_t, double, true);
        else DOCH_ADOCH_MV(int16_t, float, true);
    } else if (A.vt == ISING_F64) {
        if (!field) DOCH_ADOCH_MV(double, double, false);
        else if (A.ht == ISING_F64) DOCH_ADOCH_MV(double, double, true);
        else DOCH_ADOCH_MV(double, float, true);
    } else {
        if (!field) DOCH_ADOCH_MV(float, float, false);
        else if (A.ht == ISING_F64) DOCH_ADOCH_MV(float, double, true);
        else DOCH_ADOCH_MV(float, float, true);
    }
#undef DOCH_ADOCH_MV
    return hipGetLastError();
}

hipError_t launch_adoch_update(int64_t np, const double* x, const double* xp, const double* z,
                               const double* zp, double* xn, const AdochArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(adoch_update_kernel, dim3(grid_rows(np)), dim3(NT), 0, s, np, x, xp, z, zp, xn, a);
    return hipGetLastError();
}

hipError_t launch_adoch_finish(const double* b0, const double* b1, const double* b2,
                               const RestartState* st, int64_t n, int64_t np, bool field,
                               double* x_out, int8_t* s_out, hipStream_t s) {
    hipLaunchKernelGGL(adoch_finish_kernel, dim3(grid_rows(np)), dim3(NT), 0, s, b0, b1, b2, st, n, np,
                       field ? 1 : 0, x_out, s_out);
    return hipGetLastError();
}

}  // namespace doch
