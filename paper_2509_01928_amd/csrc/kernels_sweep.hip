// kernels_sweep.hip -- an eta sweep (Supp. Note 6) as restarts of one pass:
// up to 8 probe runs of the same CSR problem from the same start, each with
// its own alpha and beta (eq:alphabeta), iterate stored restart-interleaved
// (row i's R values contiguous, FP64), so an iteration reads the couplings,
// offsets and field once for all of them and every coupling gathers one
// 8R-byte run of the iterate.
//
// Per row and restart the arithmetic is that of the single-restart step
// (entries in ascending column order from 0.0, the field term last, then
// eq:FPE in the same expression order), so each probe's trajectory is the
// one ising_solve computes for its parameters.  The last workgroup of a
// launch finishes H, r and, with a field, the extra spin t of every restart
// (eq:Hamilton, Remark S2, Supp. Note 1).
#include "device_common.h"
#include "ising_internal.h"

#include <type_traits>
#include "step_common.h"

namespace doch {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;

// End of a sweep launch: add each restart's partial sums over the lanes that
// hold it (lanes r, r + 8, ... of a wavefront), the wavefronts and then the
// workgroups in fixed order; the last workgroup finishes H, r and, with a
// field, the extra spin t of every restart (eq:Hamilton, Remark S2, Supp.
// Note 1).
template <int R, bool FIELD>
__device__ void sweep_close(double (&acc)[kNumPartials], const SweepArgs& a, const double* __restrict__ x,
                            double* __restrict__ xn, int64_t n) {
    constexpr int G = 8;
    __shared__ double red[NW][G][kNumPartials];
    __shared__ int last_flag;
    // per restart: the wavefront's eight row groups, then the four
    // wavefronts
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) {
        double v = acc[q];
        v = dadd(v, __shfl_xor(v, 8, kWave));
        v = dadd(v, __shfl_xor(v, 16, kWave));
        v = dadd(v, __shfl_xor(v, 32, kWave));
        acc[q] = v;
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane < G)
#pragma unroll
        for (int q = 0; q < kNumPartials; ++q) red[wave][lane][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < R * kNumPartials) {
        const int rr = threadIdx.x / kNumPartials, q = threadIdx.x % kNumPartials;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s = dadd(s, red[w][rr][q]);
        store_agent(a.partials + static_cast<size_t>(blockIdx.x) * kNumPartials * R + threadIdx.x, s);
    }
    // the storing wavefront (0) waits for its stores inside the arrival
    if (threadIdx.x == 0) last_flag = arrive_last_grid(a.tickets, gridDim.x) ? 1 : 0;
    __syncthreads();
    if (!last_flag) return;
    // last workgroup: thread (r, q) of the first kNumPartials * R threads adds
    // quantity q of restart r over the workgroups in index order
    const int slot = threadIdx.x;
    double s = 0.0;
    if (slot < kNumPartials * R)
        for (unsigned g = 0; g < gridDim.x; ++g)
            s = dadd(s, load_agent(a.partials + static_cast<size_t>(g) * kNumPartials * R + slot));
    __shared__ double tot[kNumPartials * R];
    if (slot < kNumPartials * R) tot[slot] = s;
    __syncthreads();
    if (threadIdx.x >= R) return;
    const int rr = threadIdx.x;
    const double* S = tot + kNumPartials * rr;
    double S4 = S[P_X4], S2 = S[P_X2], Sxz = S[P_XZ], Sd = S[P_DX2];
    if (FIELD) {
        const double t = x[n * R + rr];
        const double zn = S[P_HX];
        const double t2 = dmul(t, t);
        S4 = dadd(S4, dmul(t2, t2));
        S2 = dadd(S2, t2);
        Sxz = dadd(Sxz, dmul(t, zn));
        const double tn = cbrt(ddiv(dadd(zn, dmul(a.alpha[rr], t)), a.beta[rr]));
        xn[n * R + rr] = tn;
        const double d = dsub(tn, t);
        Sd = dadd(Sd, dmul(d, d));
    }
    const double H = dsub(dsub(dmul(ddiv(a.beta[rr], 4.0), S4), dmul(ddiv(a.alpha[rr], 2.0), S2)), dmul(0.5, Sxz));
    const double rv = (S2 == 0.0) ? 0.0 : ddiv(sqrt(Sd), sqrt(S2));
    RestartState* st = a.state + rr;
    st->iters_done = a.k + 1;
    st->H_last = H;
    st->r_last = rv;
    if (!isfinite(H) || !isfinite(rv)) st->nonfinite = 1;
    if (rr == 0) reset_ticket(a.tickets);
}


// Eight lanes per row, lane r of the group holding restart r (lanes r >= R
// idle), so a row's R iterate values are one contiguous run of 8R bytes for
// every gather and store; the group reads the row's entries together (one
// address per load instruction and group).
template <typename VT, typename HT, bool FIELD, int R, int RL>
__global__ __launch_bounds__(NT) void csr_sweep_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const VT* __restrict__ val, const HT* __restrict__ h,
                                                       SweepArgs a) {
    constexpr int G = 8;                        // lanes per row
    const double* __restrict__ x = a.x_old;
    double* __restrict__ xn = a.x_new;
    const int r = threadIdx.x & (G - 1);
    const bool on = r < R;
    const double t_old = (FIELD && on) ? x[n * R + r] : 0.0;
    const double alpha = on ? a.alpha[r] : 1.0, beta = on ? a.beta[r] : 1.0;
    double acc[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;
    const int64_t rows_per_pass = static_cast<int64_t>(gridDim.x) * (NT / G);
    const int64_t first = static_cast<int64_t>(blockIdx.x) * (NT / G) + threadIdx.x / G;
    // row i's update from z = (J x)_i for this lane's restart
    auto update = [&](int64_t i, double z, double xi, double hq) {
        if (FIELD) z = dadd(z, dmul(hq, t_old));
        const double xnew = cbrt(ddiv(dadd(z, dmul(alpha, xi)), beta));
        xn[i * R + r] = xnew;
        const double d = dsub(xnew, xi);
        const double x2 = dmul(xi, xi);
        acc[P_X4] = dadd(acc[P_X4], dmul(x2, x2));
        acc[P_X2] = dadd(acc[P_X2], x2);
        acc[P_XZ] = dadd(acc[P_XZ], dmul(xi, z));
        acc[P_DX2] = dadd(acc[P_DX2], dmul(d, d));
        if (FIELD) acc[P_HX] = dadd(acc[P_HX], dmul(hq, xi));
    };
    if constexpr (RL == 4) {
        // rows of 4 entries at 4 i: the group reads a row's indices and
        // values as one 16-byte chunk each, two rows in flight per group
        constexpr int U = 2;
        for (int64_t base = first; base < n; base += U * rows_per_pass) {
            typename Vec4<int>::type cv[U];
            typename Vec4<VT>::type vv[U];
            double xi[U], hq[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * rows_per_pass;
                if (i < n) {
                    cv[u] = ld_stream4(col + 4 * i);
                    vv[u] = ld_stream4(val + 4 * i);
                    xi[u] = on ? x[i * R + r] : 0.0;
                    hq[u] = FIELD ? static_cast<double>(h[i]) : 0.0;
                }
            }
            double g[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * rows_per_pass;
                if (i < n && on) {
                    g[u][0] = x[static_cast<int64_t>(cv[u].x) * R + r];
                    g[u][1] = x[static_cast<int64_t>(cv[u].y) * R + r];
                    g[u][2] = x[static_cast<int64_t>(cv[u].z) * R + r];
                    g[u][3] = x[static_cast<int64_t>(cv[u].w) * R + r];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * rows_per_pass;
                if (i < n && on) {
                    const double v[4] = {static_cast<double>(vv[u].x), static_cast<double>(vv[u].y),
                                         static_cast<double>(vv[u].z), static_cast<double>(vv[u].w)};
                    double z = 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) z = dadd(z, dmul(v[q], g[u][q]));
                    update(i, z, xi[u], hq[u]);
                }
            }
        }
    } else {
        for (int64_t i = first; i < n; i += rows_per_pass) {
            double z = 0.0;
            const int e1 = rp[i + 1];
            for (int e = rp[i]; e < e1; ++e) {
                const double v = static_cast<double>(val[e]);
                const double g = on ? x[static_cast<int64_t>(col[e]) * R + r] : 0.0;
                z = dadd(z, dmul(v, g));
            }
            if (!on) continue;
            update(i, z, x[i * R + r], FIELD ? static_cast<double>(h[i]) : 0.0);
        }
    }
    sweep_close<R, FIELD>(acc, a, x, xn, n);
}

// The sweep on procedural couplings J_ij = sin(i j + seed) (0-based, zero
// diagonal, no field): each wavefront forms four rows at a time, each lane
// advancing the rows' sines along j = lane, lane + 64, ... by a rotation
// (the arguments form an arithmetic progression with step 64 i) with an
// exact sin/cos restart every 32 steps -- the step kernel's generator -- and
// every generated coupling serves all R probes: the lane loads the R
// interleaved iterate values of column j once.  Lane 8 r + q then updates
// row i0 + r of probe q.  Each probe's row sum runs in the step kernel's
// order with its couplings, so its iterates are those of a single-restart
// solve.
template <int R>
__global__ __launch_bounds__(NT) void dense_sin_sweep_kernel(int64_t n, double seed, SweepArgs a) {
    constexpr int RW = 4, U = 8, RESTART = 32;
    const double* __restrict__ x = a.x_old;
    double* __restrict__ xn = a.x_new;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double acc[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;
    for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * NW + wave) * RW; i0 < n;
         i0 += static_cast<int64_t>(gridDim.x) * NW * RW) {
        double di[RW], sd[RW], cd[RW], sv[RW], cv[RW], p[RW][R];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            di[r] = static_cast<double>(i0 + r);
            sincos(dmul(64.0, di[r]), &sd[r], &cd[r]);
            sv[r] = cv[r] = 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) p[r][q] = 0.0;
        }
        auto restart = [&](int64_t jj) {
#pragma unroll
            for (int r = 0; r < RW; ++r) sincos(dadd(dmul(di[r], static_cast<double>(jj)), seed), &sv[r], &cv[r]);
        };
        auto step = [&](int64_t jj, bool maybe_diag) {
            double xr[R];
#pragma unroll
            for (int q = 0; q < R; ++q) xr[q] = x[jj * R + q];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const double jv = (maybe_diag && jj == i0 + r) ? 0.0 : sv[r];
#pragma unroll
                for (int q = 0; q < R; ++q) p[r][q] = dadd(p[r][q], dmul(jv, xr[q]));
            }
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const double sn = fma(sv[r], cd[r], cv[r] * sd[r]);
                cv[r] = fma(cv[r], cd[r], -(sv[r] * sd[r]));
                sv[r] = sn;
            }
        };
        int64_t j = lane;
        int batch = 0;
        for (; j + (U - 1) * kWave < n; j += U * kWave, ++batch) {
            if ((batch & (RESTART / U - 1)) == 0) restart(j);
            const bool maybe_diag = i0 + RW - 1 >= j && i0 <= j + (U - 1) * kWave;
#pragma unroll
            for (int u = 0; u < U; ++u) step(j + u * kWave, maybe_diag);
        }
        for (int u = 0; j < n; j += kWave, ++u) {
            if (u == 0 && (batch & (RESTART / U - 1)) == 0) restart(j);
            step(j, true);
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double z = __shfl(wave_sum(p[r][q]), 0, kWave);
                const int64_t i = i0 + r;
                if (lane == 8 * r + q && i < n) {
                    const double xi = x[i * R + q];
                    const double xnew = cbrt(ddiv(dadd(z, dmul(a.alpha[q], xi)), a.beta[q]));
                    xn[i * R + q] = xnew;
                    const double d = dsub(xnew, xi);
                    const double x2 = dmul(xi, xi);
                    acc[P_X4] = dadd(acc[P_X4], dmul(x2, x2));
                    acc[P_X2] = dadd(acc[P_X2], x2);
                    acc[P_XZ] = dadd(acc[P_XZ], dmul(xi, z));
                    acc[P_DX2] = dadd(acc[P_DX2], dmul(d, d));
                }
            }
        }
    }
    sweep_close<R, false>(acc, a, x, xn, n);
}

// x0 (n' values) -> R interleaved copies
__global__ __launch_bounds__(NT) void sweep_load_kernel(const double* __restrict__ x0, int64_t np, int R,
                                                        double* __restrict__ X) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < np * R;
         t += static_cast<int64_t>(gridDim.x) * NT)
        X[t] = x0[t / R];
}

// spins of every restart: s_ir = sign(x_ir), times sign(t_r) with a field
__global__ __launch_bounds__(NT) void sweep_round_kernel(const double* __restrict__ X, int64_t n, int R, int field,
                                                         int8_t* __restrict__ S) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < n * R;
         t += static_cast<int64_t>(gridDim.x) * NT) {
        const int r = static_cast<int>(t % R);
        int s = X[t] >= 0.0 ? 1 : -1;
        if (field && !(X[n * R + r] >= 0.0)) s = -s;
        S[t] = static_cast<int8_t>(s);
    }
}

int grid_for(int64_t count) {
    int64_t g = (count + NT - 1) / NT;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

// eight lanes per row: 32 rows per workgroup
int grid_rows8(int64_t n) {
    int64_t g = (n + NT / 8 - 1) / (NT / 8);
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

// the 8-bit copy of the values is only streamed on 4-entry rows
template <typename VT, typename HT, bool FIELD, int RR>
void sweep_go(const CsrView& A, int grid, const SweepArgs& a, hipStream_t s) {
    const VT* v = static_cast<const VT*>(A.val);
    const HT* h = static_cast<const HT*>(A.h);
    if constexpr (std::is_same<VT, int8_t>::value) {
        hipLaunchKernelGGL((csr_sweep_kernel<VT, HT, FIELD, RR, 4>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, a);
    } else if (A.row_len == 4) {
        hipLaunchKernelGGL((csr_sweep_kernel<VT, HT, FIELD, RR, 4>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, a);
    } else {
        hipLaunchKernelGGL((csr_sweep_kernel<VT, HT, FIELD, RR, 0>), dim3(grid), dim3(NT), 0, s, A.n, A.rp,
                           A.col, v, h, a);
    }
}

template <typename VT, typename HT, bool FIELD>
hipError_t launch_sweep_f(const CsrView& A, const SweepArgs& a, hipStream_t s) {
    int grid = sweep_grid(A.n);
    if (A.row_len == 4) {
        // rows of 4 entries with implicit offsets (no dependent load chain to
        // hide) stream best with four workgroups per compute unit (measured
        // on the 10^8-spin lattice, 8 probes: 78.9 ms per sweep against 95.8
        // with 16 per CU, 87.0 with 8 and 87.6 with 2; with the 8-bit value
        // copy 74.6 ms against 73.9 with 3, 82.9 with 8, 87.4 with 2).  The
        // 16-bit column offsets are not used here: decoding them in all
        // eight lanes of a row cost more than the bytes saved (79.2 against
        // 74.8 ms per sweep on one box)
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0 &&
            grid > 4 * cus)
            grid = 4 * cus;
    }
    switch (a.R) {
#define DOCH_SWEEP_R(RR)                          \
    case RR:                                      \
        sweep_go<VT, HT, FIELD, RR>(A, grid, a, s); \
        break;
        DOCH_SWEEP_R(1)
        DOCH_SWEEP_R(2)
        DOCH_SWEEP_R(3)
        DOCH_SWEEP_R(4)
        DOCH_SWEEP_R(5)
        DOCH_SWEEP_R(6)
        DOCH_SWEEP_R(7)
        DOCH_SWEEP_R(8)
#undef DOCH_SWEEP_R
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename VT, typename HT>
hipError_t launch_sweep_v(const CsrView& A, const SweepArgs& a, hipStream_t s) {
    if (A.h) return launch_sweep_f<VT, HT, true>(A, a, s);
    return launch_sweep_f<VT, HT, false>(A, a, s);
}

}  // namespace

int sweep_grid(int64_t n) { return grid_rows8(n); }

// four rows per wavefront, 16 per workgroup
int dense_sweep_grid(int64_t n) {
    int64_t g = (n + 15) / 16;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

hipError_t launch_dense_sin_sweep(int64_t n, double seed, const SweepArgs& a, hipStream_t s) {
    const int grid = dense_sweep_grid(n);
    switch (a.R) {
#define DOCH_DSWEEP_R(RR)                                                                             \
    case RR:                                                                                          \
        hipLaunchKernelGGL((dense_sin_sweep_kernel<RR>), dim3(grid), dim3(NT), 0, s, n, seed, a);    \
        break;
        DOCH_DSWEEP_R(2)
        DOCH_DSWEEP_R(3)
        DOCH_DSWEEP_R(4)
        DOCH_DSWEEP_R(5)
        DOCH_DSWEEP_R(6)
        DOCH_DSWEEP_R(7)
        DOCH_DSWEEP_R(8)
#undef DOCH_DSWEEP_R
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_step(const CsrView& A, const SweepArgs& a, hipStream_t s) {
    const bool h64 = A.h && A.ht == ISING_F64;
    // small-integer couplings on 4-entry rows: stream the library's exact
    // 8-bit copy of the values (a quarter of the FP32 bytes)
    if (A.val8 && A.row_len == 4) {
        CsrView B = A;
        B.val = A.val8;
        return h64 ? launch_sweep_v<int8_t, double>(B, a, s) : launch_sweep_v<int8_t, float>(B, a, s);
    }
    if (A.vt == ISING_I16) return h64 ? launch_sweep_v<int16_t, double>(A, a, s) : launch_sweep_v<int16_t, float>(A, a, s);
    if (A.vt == ISING_F64) return h64 ? launch_sweep_v<double, double>(A, a, s) : launch_sweep_v<double, float>(A, a, s);
    return h64 ? launch_sweep_v<float, double>(A, a, s) : launch_sweep_v<float, float>(A, a, s);
}

hipError_t launch_sweep_load(const double* x0, int64_t np, int R, double* X, hipStream_t s) {
    hipLaunchKernelGGL(sweep_load_kernel, dim3(grid_for(np * R)), dim3(NT), 0, s, x0, np, R, X);
    return hipGetLastError();
}

hipError_t launch_sweep_round(const double* X, int64_t n, int R, bool field, int8_t* S, hipStream_t s) {
    hipLaunchKernelGGL(sweep_round_kernel, dim3(grid_for(n * R)), dim3(NT), 0, s, X, n, R, field ? 1 : 0, S);
    return hipGetLastError();
}

}  // namespace doch
