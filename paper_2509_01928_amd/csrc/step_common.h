// step_common.h -- the per-spin convexified update of eq:FPE and the
// end-of-iteration reduction (eq:Hamilton, Remark S2, extra field spin of
// Supp. Note 1) shared by the sparse and dense DOCH step kernels.
#pragma once

#include "device_common.h"
#include "ising_internal.h"

namespace doch {

// Per-thread running sums of one iteration (indices into acc[]).
enum { P_X4 = 0, P_X2 = 1, P_XZ = 2, P_DX2 = 3, P_HX = 4 };

// Row i of x^(k+1) = cbrt((z_i + alpha x_i) / beta) (eq:FPE), where z_i is
// row i of Jhat x^(k) -- the couplings plus, with a field, h_i t.  The
// expression is evaluated in exactly this order in FP64.  The new value is
// stored in the iterate's storage type and the step uses the stored value.
template <typename XT>
__device__ __forceinline__ void update_row(double z, double xi, double hi,
                                           bool field, const StepArgs& a,
                                           XT* x_new, int64_t i,
                                           double (&acc)[kNumPartials]) {
    double y = ddiv(dadd(z, dmul(a.alpha, xi)), a.beta);
    double xn = cbrt(y);
    XT xs = static_cast<XT>(xn);
    // streamed out past the caches: the next read of it is an iteration away
    __builtin_nontemporal_store(xs, x_new + i);
    double d = dsub(static_cast<double>(xs), xi);
    double x2 = dmul(xi, xi);
    acc[P_X4] = dadd(acc[P_X4], dmul(x2, x2));
    acc[P_X2] = dadd(acc[P_X2], x2);
    acc[P_XZ] = dadd(acc[P_XZ], dmul(xi, z));
    acc[P_DX2] = dadd(acc[P_DX2], dmul(d, d));
    if (field) acc[P_HX] = dadd(acc[P_HX], dmul(hi, xi));
}

// Reduce the workgroup's sums; the last workgroup to finish reduces all of
// them in a fixed order and closes the iteration:
//   H(x^(k)) = beta/4 S4 - alpha/2 S2 - 1/2 S_xz        (eq:Hamilton)
//   r^(k)    = sqrt(S_dx2) / sqrt(S2)                   (Remark S2)
// With a field the extra spin t is row n of Jhat: z_n = sum_i h_i x_i,
// t^(k+1) = cbrt((z_n + alpha t) / beta), and t enters every sum.
template <typename XT, int NT>
__device__ void step_epilogue(const StepArgs& a, double (&acc)[kNumPartials],
                              double* lds, int64_t n, bool field, double t_old) {
    __shared__ int last_flag;
    block_sum<kNumPartials, NT>(acc, lds);
    if (threadIdx.x == 0) {
        double* p = a.partials + static_cast<size_t>(blockIdx.x) * kNumPartials;
#pragma unroll
        for (int q = 0; q < kNumPartials; ++q) store_agent(p + q, acc[q]);
        last_flag = arrive_last_grid(a.ticket, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double v[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) v[q] = 0.0;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT) {
#pragma unroll
        for (int q = 0; q < kNumPartials; ++q)
            v[q] = dadd(v[q], load_agent(a.partials + static_cast<size_t>(g) * kNumPartials + q));
    }
    block_sum<kNumPartials, NT>(v, lds);
    if (threadIdx.x != 0) return;
    double S4 = v[P_X4], S2 = v[P_X2], Sxz = v[P_XZ], Sd = v[P_DX2];
    if (field) {
        const double t = t_old;
        const double zn = v[P_HX];
        const double t2 = dmul(t, t);
        S4 = dadd(S4, dmul(t2, t2));
        S2 = dadd(S2, t2);
        Sxz = dadd(Sxz, dmul(t, zn));
        double tn = cbrt(ddiv(dadd(zn, dmul(a.alpha, t)), a.beta));
        XT ts = static_cast<XT>(tn);
        static_cast<XT*>(a.x_new)[n] = ts;
        double d = dsub(static_cast<double>(ts), t);
        Sd = dadd(Sd, dmul(d, d));
    }
    double H = dsub(dsub(dmul(ddiv(a.beta, 4.0), S4), dmul(ddiv(a.alpha, 2.0), S2)),
                    dmul(0.5, Sxz));
    double r = (S2 == 0.0) ? 0.0 : ddiv(sqrt(Sd), sqrt(S2));
    a.log[2 * a.k] = H;
    a.log[2 * a.k + 1] = r;
    RestartState* st = a.state;
    st->iters_done = a.k + 1;
    st->H_last = H;
    st->r_last = r;
    if (!isfinite(H) || !isfinite(r)) {
        st->nonfinite = 1;
        st->done = 1;
    } else if (a.eps > 0.0 && r < a.eps) {
        st->converged = 1;
        st->done = 1;
    }
    // every workgroup has stopped claiming blocks: rearm the counters
    if (a.sched)
        for (int c = 0; c < 8; ++c) reset_ticket(a.sched + c * kSchedStride);
    reset_ticket(a.ticket);
}

}  // namespace doch
