// kernels_common.hip -- small elementwise kernels around the DOCH loop:
// loading the start vectors, resetting the per-restart state, the final
// sign rounding (Alg. 1 return line, with Prop. S1 for a field) and the
// normalisation step of the power iteration.
#include "device_common.h"
#include "ising_internal.h"

namespace doch {

namespace {

constexpr int NT = 256;

int grid_for(int64_t count) {
    int64_t g = (count + NT - 1) / NT;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

template <typename XT>
__global__ __launch_bounds__(NT) void load_x0_kernel(const double* __restrict__ x0,
                                                     XT* __restrict__ x, int64_t count) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < count;
         t += static_cast<int64_t>(gridDim.x) * NT)
        x[t] = static_cast<XT>(x0[t]);
}

__global__ void init_state_kernel(RestartState* st, int R, unsigned int* ticket,
                                  unsigned int* sched) {
    if (sched && threadIdx.x < 8) sched[threadIdx.x * kSchedStride] = 0u;
    // per-restart counters and the counters of a grouped grid ticket
    const int nt = R > kGridTickets ? R : kGridTickets;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) ticket[t] = 0u;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        st[r].iters_done = 0;
        st[r].done = 0;
        st[r].converged = 0;
        st[r].nonfinite = 0;
        st[r].aborted = 0;
        st[r].H_last = 0.0;
        st[r].r_last = 0.0;
    }
}

// The iterate of restart r after iters_done steps sits in buffer
// iters_done mod 2 (buffers alternate every iteration, and a stopped
// restart is never written again), or mod 3 when three buffers rotate.
template <typename XT>
__global__ __launch_bounds__(NT) void finish_kernel(const XT* __restrict__ xb0,
                                                    const XT* __restrict__ xb1,
                                                    const XT* __restrict__ xb2,
                                                    const RestartState* __restrict__ st,
                                                    int64_t n, int64_t np, int R, int field,
                                                    double* __restrict__ x_out,
                                                    int8_t* __restrict__ s_out) {
    const int64_t total = np * R;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * NT) {
        const int64_t i = t / R;
        const int r = static_cast<int>(t - i * R);
        const int64_t m = xb2 ? st[r].iters_done % 3 : (st[r].iters_done & 1);
        const XT* xb = m == 0 ? xb0 : (m == 1 ? xb1 : xb2);
        const double x = static_cast<double>(xb[t]);
        if (x_out) x_out[t] = x;
        if (s_out && i < n) {
            int s = (x >= 0.0) ? 1 : -1;
            if (field) {
                const double tv = static_cast<double>(xb[n * R + r]);
                if (!(tv >= 0.0)) s = -s;
            }
            s_out[t] = static_cast<int8_t>(s);
        }
    }
}

__global__ __launch_bounds__(NT) void normalize_kernel(const double* __restrict__ w,
                                                       double* __restrict__ v,
                                                       const double* __restrict__ mu_log,
                                                       int64_t k, int64_t n) {
    const double nrm = mu_log[2 * k + 1];
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < n;
         t += static_cast<int64_t>(gridDim.x) * NT)
        v[t] = ddiv(w[t], nrm);
}

// Supp. Note 5 with w = -J: cut = -S_J / 4 - E / 2 (exact in int64 for
// integer couplings, where S_J + 2 E is a multiple of 4).
__global__ void cut_kernel(const double* __restrict__ E, const int64_t* __restrict__ E_int,
                           const MatrixStats* __restrict__ ms, int R, double* __restrict__ cut,
                           int64_t* __restrict__ cut_int) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double s1 = ms->s1;
    if (cut) cut[r] = dsub(dmul(-0.25, s1), dmul(0.5, E[r]));
    if (cut_int) cut_int[r] = -(llround(s1) + 2 * E_int[r]) / 4;
}

}  // namespace

hipError_t launch_cut(const double* E, const int64_t* E_int, const MatrixStats* ms, int R, double* cut,
                      int64_t* cut_int, hipStream_t s) {
    hipLaunchKernelGGL(cut_kernel, dim3((R + 255) / 256), dim3(256), 0, s, E, E_int, ms, R, cut, cut_int);
    return hipGetLastError();
}

hipError_t launch_load_x0(const double* x0, void* x, int x_dtype, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (x_dtype == ISING_F64)
        hipLaunchKernelGGL(load_x0_kernel<double>, dim3(grid_for(count)), dim3(NT), 0, s, x0,
                           static_cast<double*>(x), count);
    else
        hipLaunchKernelGGL(load_x0_kernel<float>, dim3(grid_for(count)), dim3(NT), 0, s, x0,
                           static_cast<float*>(x), count);
    return hipGetLastError();
}

hipError_t launch_init_state(RestartState* st, int R, unsigned int* ticket, unsigned int* sched,
                             hipStream_t s) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st, R, ticket, sched);
    return hipGetLastError();
}

hipError_t launch_finish(const void* xb0, const void* xb1, const void* xb2, int x_dtype, const RestartState* st,
                         int64_t n, int64_t np, int R, bool field, double* x_out, int8_t* s_out,
                         hipStream_t s) {
    const int grid = grid_for(np * R);
    if (x_dtype == ISING_F64)
        hipLaunchKernelGGL(finish_kernel<double>, dim3(grid), dim3(NT), 0, s,
                           static_cast<const double*>(xb0), static_cast<const double*>(xb1),
                           static_cast<const double*>(xb2), st, n,
                           np, R, field ? 1 : 0, x_out, s_out);
    else
        hipLaunchKernelGGL(finish_kernel<float>, dim3(grid), dim3(NT), 0, s,
                           static_cast<const float*>(xb0), static_cast<const float*>(xb1),
                           static_cast<const float*>(xb2), st, n,
                           np, R, field ? 1 : 0, x_out, s_out);
    return hipGetLastError();
}

hipError_t launch_normalize(const double* w, double* v, const double* mu_log, int64_t k,
                            int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(n)), dim3(NT), 0, s, w, v, mu_log, k, n);
    return hipGetLastError();
}

}  // namespace doch
