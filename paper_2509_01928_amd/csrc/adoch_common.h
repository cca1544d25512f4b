// adoch_common.h -- the closing step of an ADOCH (Alg. 2) matvec launch,
// shared by the CSR and dense kernels.
//
// Iteration k of R interleaved restarts: every workgroup has added, per
// restart, x^4, x^2, x.z, y^4, y^2, y.(J y) and h.x over its rows, with
// y = x^(k) + c_k (x^(k) - x^(k-1)) and J y = (1 + c_k) z_k - c_k z_{k-1}
// (one matvec per iteration, by linearity).  The last workgroup adds the
// workgroups' sums in workgroup order, closes the field spin's row, forms
// H(x^(k)) and H(y^(k)) (eq:Hamilton), keeps the window of the last q + 1
// values of H(x) and decides per restart whether y is taken (H(y) at most
// the window's maximum, eq:BBscheme).
#pragma once

#include "device_common.h"
#include "ising_internal.h"

namespace doch {

// Store this workgroup's S R sums and, in the last workgroup to arrive,
// close the iteration.  acc: thread 0's workgroup totals (restart r at S r,
// S = 7, or 8 with OPT).
//
// OPT (the CSR product that has already written x^(k+1) = T(y^(k)) for every
// restart that had not stopped, and copied stopped ones forward): the eighth
// sum is |T(y) - x^(k)|^2, so an accepted restart is closed here, r^(k)
// and Remark S2's test included.  A rejected restart is left to the fix-up
// launch (fix[r] = 1: x^(k+1) = T(x^(k)) recomputed), so is one whose H(x)
// is not finite (fix[r] = 2: x^(k) copied forward); fix[8] says whether any
// is pending, and all_done is raised here only when none is.
template <int R, int NT, bool FIELD, bool OPT = false>
__device__ __forceinline__ void adoch_mv_close(double (&acc)[(OPT ? 8 : 7) * R], double* red, int* last_flag,
                                               int64_t n, const double* __restrict__ x,
                                               const double* __restrict__ xp, const double* __restrict__ zp,
                                               double* __restrict__ z, const AdochArgs& a,
                                               double* __restrict__ xn = nullptr) {
    constexpr int S = OPT ? 8 : 7;
    constexpr int K = S * R;
    if (threadIdx.x == 0) {
        double* p = a.partials + static_cast<size_t>(blockIdx.x) * K;
#pragma unroll
        for (int q = 0; q < K; ++q) store_agent(p + q, acc[q]);
        *last_flag = arrive_last_grid(a.ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!*last_flag) return;
    double u[K];
#pragma unroll
    for (int q = 0; q < K; ++q) u[q] = 0.0;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT)
#pragma unroll
        for (int q = 0; q < K; ++q) u[q] = dadd(u[q], load_agent(a.partials + static_cast<size_t>(g) * K + q));
    block_sum<K, NT>(u, red);
    // the totals to LDS, then one thread per restart: each restart's closing
    // is a chain of dependent global accesses (state, window, logs), so the
    // restarts run side by side instead of one after another
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) red[q] = u[q];
    __syncthreads();
    __shared__ int flags[2 * R];                // per restart: pending fix-up, stopped
    const int r = threadIdx.x;
    if (r < R) {
        const double c = a.c;
        const double b4 = ddiv(a.beta, 4.0), a2 = ddiv(a.alpha, 2.0);
        const int W = a.q + 1;
        int pending = 0;
        RestartState& st = a.state[r];
        if (OPT) a.fix[r] = 0;
        if (st.done) {
            if (OPT && FIELD) xn[n * R + r] = x[n * R + r];
        } else {
            double ur[8];                       // the eighth sum only with OPT
#pragma unroll
            for (int q = 0; q < 8; ++q) ur[q] = q < S ? red[S * r + q] : 0.0;
            if (FIELD) {
                // the extra spin's row: z_n = sum_i h_i x_i, and its share of every sum
                const int64_t tn = n * R + r;
                const double tx = x[tn];
                const double zn = ur[6];
                z[tn] = zn;
                const double yn = dadd(tx, dmul(c, dsub(tx, xp[tn])));
                const double jyn = dsub(dmul(dadd(1.0, c), zn), dmul(c, zp[tn]));
                const double t2 = dmul(tx, tx), y2 = dmul(yn, yn);
                ur[0] = dadd(ur[0], dmul(t2, t2));
                ur[1] = dadd(ur[1], t2);
                ur[2] = dadd(ur[2], dmul(tx, zn));
                ur[3] = dadd(ur[3], dmul(y2, y2));
                ur[4] = dadd(ur[4], y2);
                ur[5] = dadd(ur[5], dmul(yn, jyn));
                if (OPT) {
                    const double nx = cbrt(ddiv(dadd(jyn, dmul(a.alpha, yn)), a.beta));
                    xn[tn] = nx;
                    const double d = dsub(nx, tx);
                    ur[7] = dadd(ur[7], dmul(d, d));
                }
            }
            const double Hx = dsub(dsub(dmul(b4, ur[0]), dmul(a2, ur[1])), dmul(0.5, ur[2]));
            const double Hy = dsub(dsub(dmul(b4, ur[3]), dmul(a2, ur[4])), dmul(0.5, ur[5]));
            // window of H(x^(j)), max(0, k - q) <= j <= k
            double* ring = a.ring + static_cast<size_t>(r) * W;
            ring[a.k % W] = Hx;
            const int64_t j0 = a.k - a.q > 0 ? a.k - a.q : 0;
            double hmax = Hx;
            for (int64_t j = j0; j < a.k; ++j) hmax = fmax(hmax, ring[j % W]);
            const int accept = Hy <= hmax ? 1 : 0;
            a.accept[r] = accept;
            a.log[(static_cast<size_t>(a.k) * R + r) * 2] = Hx;
            a.accept_log[static_cast<size_t>(a.k) * R + r] = static_cast<int8_t>(accept);
            st.H_last = Hx;
            if (!isfinite(Hx)) {
                st.nonfinite = 1;
                st.done = 1;
                st.iters_done = a.k + 1;
                if (OPT) {
                    a.fix[r] = 2;
                    pending = 1;
                }
            } else if (OPT && !accept) {
                a.fix[r] = 1;
                pending = 1;
            } else if (OPT) {
                const double rr = ur[1] == 0.0 ? 0.0 : ddiv(sqrt(ur[7]), sqrt(ur[1]));
                a.log[(static_cast<size_t>(a.k) * R + r) * 2 + 1] = rr;
                st.iters_done = a.k + 1;
                st.r_last = rr;
                if (!isfinite(rr)) {
                    st.nonfinite = 1;
                    st.done = 1;
                } else if (a.eps > 0.0 && rr < a.eps) {
                    st.converged = 1;
                    st.done = 1;
                }
            }
        }
        flags[r] = pending;
        flags[R + r] = st.done;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (OPT) {
        int pending = 0, all = 1;
        for (int q = 0; q < R; ++q) {
            pending |= flags[q];
            all &= flags[R + q];
        }
        a.fix[8] = pending;
        if (!pending && all) *a.all_done = 1;
    }
    reset_ticket(a.ticket);
}

}  // namespace doch
