// kernels_dense.hip -- dense FP64 kernels of the DOCH hot path for gfx950.
//
// One wavefront owns one row of J: its 64 lanes stream the row with
// unit-stride 8-byte loads (512 contiguous bytes per instruction), multiply by
// the iterate, and a butterfly reduction gives (J x)_i; lane 0 then applies
// the cube-root update of eq:FPE.  Four wavefronts (four rows) share a
// workgroup.  A single-vector FP64 product has no data reuse, so it runs on
// the vector ALUs, not on the matrix cores.  The same kernels also serve the
// procedural couplings J_ij = sin(i j + seed), generated in registers instead
// of loaded (compute-bound on FP64 sine).
#include <type_traits>

#include "adoch_common.h"
#include "device_common.h"
#include "ising_internal.h"
#include "step_common.h"

namespace doch {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;

// Where the couplings come from: a stored row-major matrix, or the
// procedural rule J_ij = sin(i j + seed) (0-based indices, zero diagonal) of
// Supp. Note 9, evaluated on demand in FP64 (i j < 2^53 is exact).
struct StoredJ {
    const double* J;
    int64_t ld;
    __device__ __forceinline__ double operator()(int64_t i, int64_t j) const { return J[i * ld + j]; }
};
struct SinJ {
    double seed;
    __device__ __forceinline__ double operator()(int64_t i, int64_t j) const {
        return i == j ? 0.0 : sin(dadd(dmul(static_cast<double>(i), static_cast<double>(j)), seed));
    }
};

// Lane's share of row i of J times a vector: sum over j = lane, lane + 64, ...
// in that order (the wavefront then adds the 64 lane sums).  Loads are issued
// eight columns at a time before they are added, so a row costs a few memory
// round trips instead of one per column.
template <typename JS, typename V>
__device__ __forceinline__ double lane_row_dot(const JS& J, int64_t i, V vec, int64_t n, int lane) {
    constexpr int U = 8;
    double p = 0.0;
    int64_t j = lane;
    for (; j + (U - 1) * kWave < n; j += U * kWave) {
        double jv[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            jv[u] = J(i, j + u * kWave);
            xv[u] = vec(j + u * kWave);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) p = dadd(p, dmul(jv[u], xv[u]));
    }
    for (; j < n; j += kWave) p = dadd(p, dmul(J(i, j), vec(j)));
    return p;
}

// Lane's share of RW consecutive rows i0 .. i0 + RW - 1 of J_ij = sin(i j +
// seed) times a vector, in the order of lane_row_dot (j = lane, lane + 64,
// ...), each loaded x_j serving all RW rows.  A row's arguments i j + seed
// along the lane form an arithmetic progression with step d = 64 i, so its
// (sin, cos) pair advances by the rotation (cos d, sin d) -- four products
// per coupling instead of a range-reduced sine -- and restarts from an exact
// sin/cos every kSinRestart steps, which bounds the accumulated rounding to
// a few dozen ulp.  All angles are integers (plus the seed) below 2^53, so
// each restart is exact to the sine's own accuracy.
constexpr int kSinRestart = 32;
template <int RW, typename V>
__device__ __forceinline__ void lane_rows_dot_sin(const SinJ& J, int64_t i0, V vec, int64_t n, int lane,
                                                  double (&p)[RW]) {
    constexpr int U = 8;                         // steps per batch; kSinRestart is 4 batches
    static_assert(kSinRestart % U == 0, "restarts fall on batch boundaries");
    double di[RW], sd[RW], cd[RW], sv[RW], cv[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        di[r] = static_cast<double>(i0 + r);
        sincos(dmul(64.0, di[r]), &sd[r], &cd[r]);
        p[r] = 0.0;
        sv[r] = cv[r] = 0.0;
    }
    auto restart = [&](int64_t jj) {
#pragma unroll
        for (int r = 0; r < RW; ++r) sincos(dadd(dmul(di[r], static_cast<double>(jj)), J.seed), &sv[r], &cv[r]);
    };
    auto rotate = [&]() {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const double sn = fma(sv[r], cd[r], cv[r] * sd[r]);
            cv[r] = fma(cv[r], cd[r], -(sv[r] * sd[r]));
            sv[r] = sn;
        }
    };
    // one coupling step of every row; the diagonal (J_ii = 0) is tested only
    // in batches that can hold it
    auto step = [&](int64_t jj, double x, bool maybe_diag) {
        if (maybe_diag) {
#pragma unroll
            for (int r = 0; r < RW; ++r) p[r] = dadd(p[r], dmul(jj == i0 + r ? 0.0 : sv[r], x));
        } else {
#pragma unroll
            for (int r = 0; r < RW; ++r) p[r] = dadd(p[r], dmul(sv[r], x));
        }
        rotate();
    };
    int64_t j = lane;
    int batch = 0;
    // full batches: all U steps in range
    for (; j + (U - 1) * kWave < n; j += U * kWave, ++batch) {
        if ((batch & (kSinRestart / U - 1)) == 0) restart(j);
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = vec(j + u * kWave);
        // the batch's steps j, j + 64, ..., j + 448 meet rows i0 .. i0 + RW - 1
        // only if those rows lie within [j, j + 448]
        const bool maybe_diag = i0 + RW - 1 >= j && i0 <= j + (U - 1) * kWave;
#pragma unroll
        for (int u = 0; u < U; ++u) step(j + u * kWave, xv[u], maybe_diag);
    }
    // the last, partial batch
    for (int u = 0; j < n; j += kWave, ++u) {
        if (u == 0 && (batch & (kSinRestart / U - 1)) == 0) restart(j);
        step(j, vec(j), true);
    }
}

// The same generator as lane_rows_dot_sin, handing each step to a visitor:
// f(j, sv, dr) sees column j, the current sines sv[r] = sin((i0 + r) j +
// seed) of the RW rows and dr = j - i0 when column j is one of the rows'
// diagonals (J_ii = 0: the visitor skips row dr there), else -1.
template <int RW, typename F>
__device__ __forceinline__ void lane_rows_sin_walk(const SinJ& J, int64_t i0, int64_t n, int lane, F&& f) {
    constexpr int U = 8;
    double di[RW], sd[RW], cd[RW], sv[RW], cv[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        di[r] = static_cast<double>(i0 + r);
        sincos(dmul(64.0, di[r]), &sd[r], &cd[r]);
        sv[r] = cv[r] = 0.0;
    }
    auto restart = [&](int64_t jj) {
#pragma unroll
        for (int r = 0; r < RW; ++r) sincos(dadd(dmul(di[r], static_cast<double>(jj)), J.seed), &sv[r], &cv[r]);
    };
    auto rotate = [&]() {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const double sn = fma(sv[r], cd[r], cv[r] * sd[r]);
            cv[r] = fma(cv[r], cd[r], -(sv[r] * sd[r]));
            sv[r] = sn;
        }
    };
    auto diag = [&](int64_t jj) { return (jj >= i0 && jj < i0 + RW) ? static_cast<int>(jj - i0) : -1; };
    int64_t j = lane;
    int batch = 0;
    for (; j + (U - 1) * kWave < n; j += U * kWave, ++batch) {
        if ((batch & (kSinRestart / U - 1)) == 0) restart(j);
        // batches that cannot hold a diagonal pass a constant -1, so the
        // visitor's test folds away there
        if (i0 + RW - 1 >= j && i0 <= j + (U - 1) * kWave) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f(j + u * kWave, sv, diag(j + u * kWave));
                rotate();
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f(j + u * kWave, sv, -1);
                rotate();
            }
        }
    }
    for (int u = 0; j < n; j += kWave, ++u) {
        if (u == 0 && (batch & (kSinRestart / U - 1)) == 0) restart(j);
        f(j, sv, diag(j));
        rotate();
    }
}

// rows of the procedural couplings a wavefront forms together
constexpr int kSinRows = 4;

template <typename XT, typename HT, bool FIELD, typename JS>
__global__ __launch_bounds__(NT) void dense_step_kernel(int64_t n, JS J,
                                                        const HT* __restrict__ h, StepArgs a) {
    if (a.state->done) return;
    __shared__ double red[kNumPartials * NW];
    const XT* __restrict__ x = static_cast<const XT*>(a.x_old);
    XT* __restrict__ xn = static_cast<XT*>(a.x_new);
    const double t_old = FIELD ? static_cast<double>(x[n]) : 0.0;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double acc[kNumPartials];
#pragma unroll
    for (int q = 0; q < kNumPartials; ++q) acc[q] = 0.0;
    auto xv = [&](int64_t j) { return static_cast<double>(x[j]); };
    if constexpr (std::is_same<JS, SinJ>::value) {
        // kSinRows rows per wavefront; lane r updates row i0 + r with the
        // row total as lane 0 forms it
        constexpr int RW = kSinRows;
        for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * NW + wave) * RW; i0 < n;
             i0 += static_cast<int64_t>(gridDim.x) * NW * RW) {
            double p[RW];
            lane_rows_dot_sin<RW>(J, i0, xv, n, lane, p);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const double z0 = __shfl(wave_sum(p[r]), 0, kWave);
                const int64_t i = i0 + r;
                if (lane == r && i < n) {
                    double z = z0;
                    double hv = 0.0;
                    if (FIELD) {
                        hv = static_cast<double>(h[i]);
                        z = dadd(z, dmul(hv, t_old));
                    }
                    update_row<XT>(z, static_cast<double>(x[i]), hv, FIELD, a, xn, i, acc);
                }
            }
        }
        step_epilogue<XT, NT>(a, acc, red, n, FIELD, t_old);
        return;
    }
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave; i < n;
         i += static_cast<int64_t>(gridDim.x) * NW) {
        double p = lane_row_dot(J, i, xv, n, lane);
        const double z0 = wave_sum(p);
        if (lane == 0) {
            double z = z0;
            double hv = 0.0;
            if (FIELD) {
                hv = static_cast<double>(h[i]);
                z = dadd(z, dmul(hv, t_old));
            }
            update_row<XT>(z, static_cast<double>(x[i]), hv, FIELD, a, xn, i, acc);
        }
    }
    step_epilogue<XT, NT>(a, acc, red, n, FIELD, t_old);
}

// eq:IsingModel for many restarts at once: Z = J S for the n x R spin block,
// 64 x 64 output tiles per workgroup, each thread a 4 x 4 block, J and S
// staged through LDS in k slices of 32, so each coupling is read (or
// generated) once per 64 restarts.  Per restart the tile adds s_i z_i and
// h_i s_i over its rows; the last workgroup of each column block adds the row
// tiles in order and writes E = -1/2 s^T J s - h^T s.
template <typename HT, bool FIELD, typename JS>
__global__ __launch_bounds__(NT) void dense_energy_tiled_kernel(int64_t n, JS J, const HT* __restrict__ h,
                                                                const int8_t* __restrict__ S, int R, int Rp,
                                                                double* __restrict__ partials,
                                                                unsigned int* tickets, double* __restrict__ E) {
    constexpr int KS = 32;
    __shared__ double Js[64][KS + 1];
    __shared__ double Ss[KS][64];
    __shared__ double cred[16][64][2];
    __shared__ int last_flag;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 64;
    const int col0 = blockIdx.y * 64;
    double acc[4][4] = {};
    for (int64_t k0 = 0; k0 < n; k0 += KS) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + NT * u;
            const int r = e / KS, kk = e % KS;
            const int64_t gi = row0 + r, gk = k0 + kk;
            Js[r][kk] = (gi < n && gk < n) ? J(gi, gk) : 0.0;
            const int sk = e / 64, sc = e % 64;
            const int64_t hk = k0 + sk;
            const int hc = col0 + sc;
            Ss[sk][sc] = (hk < n && hc < R) ? static_cast<double>(S[hk * R + hc]) : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KS; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = Js[ty * 4 + q][kk];
                b[q] = Ss[kk][tx * 4 + q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
    double v[4][2] = {};
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int64_t i = row0 + ty * 4 + p;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = col0 + tx * 4 + q;
            if (i < n && c < R) {
                const double si = static_cast<double>(S[i * R + c]);
                v[q][0] = dadd(v[q][0], dmul(si, acc[p][q]));
                if (FIELD) v[q][1] = dadd(v[q][1], dmul(static_cast<double>(h[i]), si));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        cred[ty][tx * 4 + q][0] = v[q][0];
        cred[ty][tx * 4 + q][1] = v[q][1];
    }
    __syncthreads();
    if (tid < 64) {                             // wave 0: the wave that releases below
        double* pp = partials + (static_cast<size_t>(blockIdx.x) * Rp + col0 + tid) * 2;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            double sm = 0.0;
            for (int t = 0; t < 16; ++t) sm = dadd(sm, cred[t][tid][m]);
            store_agent(pp + m, sm);
        }
    }
    __syncthreads();
    if (tid == 0) last_flag = arrive_last(tickets + blockIdx.y, gridDim.x) ? 1 : 0;
    __syncthreads();
    if (!last_flag) return;
    if (tid < 2 * 64) {
        const int cl = tid & 63, m = tid >> 6;
        cred[0][cl][m] = column_partial_sum<2>(partials, Rp, col0 + cl, m, gridDim.x);
    }
    __syncthreads();
    if (tid < 64 && col0 + tid < R) E[col0 + tid] = dsub(dmul(-0.5, cred[0][tid][0]), cred[0][tid][1]);
    if (tid == 0) reset_ticket(tickets + blockIdx.y);
}

template <typename HT, bool FIELD, typename JS>
__global__ __launch_bounds__(NT) void dense_energy_kernel(int64_t n, JS J,
                                                          const HT* __restrict__ h,
                                                          const int8_t* __restrict__ s, int R,
                                                          double* partials, unsigned int* tickets,
                                                          double* E) {
    __shared__ double red[2 * NW];
    __shared__ int last_flag;
    const int r = blockIdx.y;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double v[2] = {0.0, 0.0};
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave; i < n;
         i += static_cast<int64_t>(gridDim.x) * NW) {
        double p = 0.0;
        p = lane_row_dot(J, i, [&](int64_t j) { return static_cast<double>(s[j * R + r]); }, n, lane);
        const double z = wave_sum(p);
        if (lane == 0) {
            const double si = static_cast<double>(s[i * R + r]);
            v[0] = dadd(v[0], dmul(si, z));
            if (FIELD) v[1] = dadd(v[1], dmul(static_cast<double>(h[i]), si));
        }
    }
    block_sum<2, NT>(v, red);
    double* p = partials + (static_cast<size_t>(r) * gridDim.x + blockIdx.x) * 2;
    if (threadIdx.x == 0) {
        store_agent(p + 0, v[0]);
        store_agent(p + 1, v[1]);
        last_flag = arrive_last(tickets + r, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[2] = {0.0, 0.0};
    const double* pr = partials + static_cast<size_t>(r) * gridDim.x * 2;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += NT) {
        u[0] = dadd(u[0], load_agent(pr + g * 2 + 0));
        u[1] = dadd(u[1], load_agent(pr + g * 2 + 1));
    }
    block_sum<2, NT>(u, red);
    if (threadIdx.x == 0) {
        E[r] = dsub(dmul(-0.5, u[0]), u[1]);
        reset_ticket(tickets + r);
    }
}

// eq:IsingModel on the procedural couplings for RB restarts at once: each
// wavefront forms four rows with the step kernel's sine generator, and every
// generated coupling serves the RB restarts c0 .. c0 + RB - 1 of its column
// block (restarts beyond R are left out).  Per restart the workgroup adds
// s_i z_i over its rows; the last workgroup of a column block adds the
// workgroups' sums in index order and writes E = -1/2 s^T J s.  PACKED: a
// full block of 8 at an 8-byte aligned address, its spins of column j read
// as one 8-byte word.
template <int RB, bool PACKED>
__global__ __launch_bounds__(NT) void dense_sin_energy_kernel(int64_t n, SinJ J, const int8_t* __restrict__ S,
                                                              int R, double* partials, unsigned int* tickets,
                                                              double* E) {
    constexpr int RW = kSinRows;
    __shared__ double red[RB * NW];
    __shared__ int last_flag;
    const int c0 = blockIdx.y * RB;
    const int nc = min(RB, R - c0);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double v[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) v[q] = 0.0;
    for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * NW + wave) * RW; i0 < n;
         i0 += static_cast<int64_t>(gridDim.x) * NW * RW) {
        double p[RW][RB];
        if constexpr (RB == 1) {
            double p1[RW];
            lane_rows_dot_sin<RW>(J, i0, [&](int64_t j) { return static_cast<double>(S[j * R + c0]); }, n,
                                  lane, p1);
#pragma unroll
            for (int r = 0; r < RW; ++r) p[r][0] = p1[r];
        } else {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int q = 0; q < RB; ++q) p[r][q] = 0.0;
            lane_rows_sin_walk<RW>(J, i0, n, lane, [&](int64_t j, const double (&sv)[RW], int dr) {
                double sj[RB];
                if constexpr (PACKED) {
                    const uint64_t w = *reinterpret_cast<const uint64_t*>(S + j * R + c0);
#pragma unroll
                    for (int q = 0; q < RB; ++q) sj[q] = static_cast<double>(static_cast<int8_t>(w >> (8 * q)));
                } else {
#pragma unroll
                    for (int q = 0; q < RB; ++q) sj[q] = q < nc ? static_cast<double>(S[j * R + c0 + q]) : 0.0;
                }
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const double jv = r == dr ? 0.0 : sv[r];
#pragma unroll
                    for (int q = 0; q < RB; ++q) p[r][q] = dadd(p[r][q], dmul(jv, sj[q]));
                }
            });
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int64_t i = i0 + r;
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const double z = wave_sum(p[r][q]);
                if (lane == 0 && i < n && q < nc) v[q] = dadd(v[q], dmul(static_cast<double>(S[i * R + c0 + q]), z));
            }
        }
    }
    block_sum<RB, NT>(v, red);
    if (threadIdx.x == 0) {
        for (int q = 0; q < nc; ++q)
            store_agent(partials + static_cast<size_t>(c0 + q) * gridDim.x + blockIdx.x, v[q]);
        last_flag = arrive_last(tickets + blockIdx.y, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        u[q] = 0.0;
        if (q < nc) {
            const double* pr = partials + static_cast<size_t>(c0 + q) * gridDim.x;
            for (unsigned g = threadIdx.x; g < gridDim.x; g += NT) u[q] = dadd(u[q], load_agent(pr + g));
        }
    }
    block_sum<RB, NT>(u, red);
    if (threadIdx.x == 0) {
        for (int q = 0; q < nc; ++q) E[c0 + q] = dmul(-0.5, u[q]);
        reset_ticket(tickets + blockIdx.y);
    }
}

// flags[0]: non-finite entry, flags[1]: nonzero diagonal, flags[2]: an entry
// is not an integer of magnitude < 2^31.
__global__ __launch_bounds__(NT) void dense_validate_kernel(int64_t n, int64_t ld,
                                                            const double* __restrict__ J,
                                                            int32_t* flags) {
    const int64_t total = n * n;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * NT) {
        const int64_t i = t / n, j = t % n;
        const double v = J[i * ld + j];
        if (!isfinite(v)) atomicOr(flags + 0, 1);
        if (i == j && v != 0.0) atomicOr(flags + 1, 1);
        if (!(v == floor(v)) || fabs(v) >= 2147483648.0) atomicOr(flags + 2, 1);
    }
}

__global__ __launch_bounds__(NT) void dense_symcheck_kernel(int64_t n, int64_t ld,
                                                            const double* __restrict__ J,
                                                            int32_t* bad) {
    const int64_t total = n * n;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * NT) {
        const int64_t i = t / n, j = t % n;
        if (J[i * ld + j] != J[j * ld + i]) atomicOr(bad, 1);
    }
}

template <typename HT, bool FIELD, typename JS>
__global__ __launch_bounds__(NT) void dense_stats_kernel(int64_t n, JS J,
                                                         const HT* __restrict__ h, double mean,
                                                         int pass, double* partials,
                                                         unsigned int* ticket, MatrixStats* out) {
    __shared__ double red[3 * NW];
    __shared__ double redm[NW];
    __shared__ int last_flag;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double v[3] = {0.0, 0.0, 0.0};
    double pmax = 0.0;
    // row i's sums over j != i: rs of |J_ij| (pass 0) or (J_ij - mean)^2
    // (pass 1), sm of J_ij, complete in lane 0
    auto row_done = [&](int64_t i, double rs, double sm) {
        if (lane == 0) {
            if (pass == 0) {
                double rsum = rs;
                v[0] = dadd(v[0], sm);
                v[1] += static_cast<double>(n - 1);
                if (FIELD) {
                    const double hv = static_cast<double>(h[i]);
                    rsum = dadd(rsum, fabs(hv));
                    v[0] = dadd(v[0], dmul(2.0, hv));
                    v[1] += 2.0;
                    v[2] = dadd(v[2], fabs(hv));
                }
                pmax = fmax(pmax, rsum);
            } else {
                v[0] = dadd(v[0], rs);
                if (FIELD) {
                    const double d = dsub(static_cast<double>(h[i]), mean);
                    v[0] = dadd(v[0], dmul(2.0, dmul(d, d)));
                }
            }
        }
    };
    auto add = [&](double& a0, double& a1, double x) {
        if (pass == 0) {
            a0 = dadd(a0, fabs(x));
            a1 = dadd(a1, x);
        } else {
            const double d = dsub(x, mean);
            a0 = dadd(a0, dmul(d, d));
        }
    };
    if constexpr (std::is_same<JS, SinJ>::value) {
        // kSinRows rows per wavefront from the sine generator, one walk per
        // pass so that the loop holds only that pass's arithmetic
        constexpr int RW = kSinRows;
        for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * NW + wave) * RW; i0 < n;
             i0 += static_cast<int64_t>(gridDim.x) * NW * RW) {
            double a0[RW], a1[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) a0[r] = a1[r] = 0.0;
            if (pass == 0) {
                lane_rows_sin_walk<RW>(J, i0, n, lane, [&](int64_t, const double (&sv)[RW], int dr) {
#pragma unroll
                    for (int r = 0; r < RW; ++r)
                        if (r != dr) {
                            a0[r] = dadd(a0[r], fabs(sv[r]));
                            a1[r] = dadd(a1[r], sv[r]);
                        }
                });
            } else {
                lane_rows_sin_walk<RW>(J, i0, n, lane, [&](int64_t, const double (&sv)[RW], int dr) {
#pragma unroll
                    for (int r = 0; r < RW; ++r)
                        if (r != dr) {
                            const double d = dsub(sv[r], mean);
                            a0[r] = dadd(a0[r], dmul(d, d));
                        }
                });
            }
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const double rs = wave_sum(a0[r]);
                const double sm = wave_sum(a1[r]);
                if (i0 + r < n) row_done(i0 + r, rs, sm);
            }
        }
    } else {
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave; i < n;
             i += static_cast<int64_t>(gridDim.x) * NW) {
            double a0 = 0.0, a1 = 0.0;
            for (int64_t j = lane; j < n; j += kWave) {
                if (j == i) continue;
                add(a0, a1, J(i, j));
            }
            const double rs = wave_sum(a0);
            const double sm = wave_sum(a1);
            row_done(i, rs, sm);
        }
    }
    block_sum<3, NT>(v, red);
    const double wm = wave_max(pmax);
    if (lane == 0) redm[wave] = wm;
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
    const double wum = wave_max(um);
    if (lane == 0) redm[wave] = wum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < NW; ++w) m = fmax(m, redm[w]);
        if (pass == 0) {
            const double rmax = FIELD ? fmax(m, u[2]) : m;
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

template <typename HT, bool FIELD, typename JS>
__global__ __launch_bounds__(NT) void dense_power_kernel(int64_t n, JS J,
                                                         const HT* __restrict__ h, double c,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ w, double* partials,
                                                         unsigned int* ticket, double* mu_log,
                                                         int64_t k) {
    __shared__ double red[3 * NW];
    __shared__ int last_flag;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const double vn = FIELD ? v[n] : 0.0;
    double acc[3] = {0.0, 0.0, 0.0};
    // w_i = c v_i - (J v)_i from row i's total z0, in lane 0
    auto row_done = [&](int64_t i, double z0) {
        if (lane == 0) {
            double z = z0;
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
    };
    auto vv = [&](int64_t j) { return v[j]; };
    if constexpr (std::is_same<JS, SinJ>::value) {
        // kSinRows rows per wavefront from the sine generator
        constexpr int RW = kSinRows;
        for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * NW + wave) * RW; i0 < n;
             i0 += static_cast<int64_t>(gridDim.x) * NW * RW) {
            double p[RW];
            lane_rows_dot_sin<RW>(J, i0, vv, n, lane, p);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const double z0 = wave_sum(p[r]);
                if (i0 + r < n) row_done(i0 + r, z0);
            }
        }
    } else {
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave; i < n;
             i += static_cast<int64_t>(gridDim.x) * NW)
            row_done(i, wave_sum(lane_row_dot(J, i, vv, n, lane)));
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

// ADOCH (Alg. 2) matvec of R interleaved restarts on dense couplings: z =
// Jhat x^(k) with the sums of H(x^(k)) and H(y^(k)) (see adoch_common.h).
// Stored J: a wavefront per row, each loaded J_ij serving the R restarts;
// generated J: kSinRows rows per wavefront, each generated sine serving the
// R restarts of its row.  Rows are summed in the column order of the DOCH
// step kernels.
template <typename HT, bool FIELD, typename JS, int R>
__global__ __launch_bounds__(NT) void adoch_dense_mv_kernel(int64_t n, JS J, const HT* __restrict__ h,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ xp,
                                                            const double* __restrict__ zp, double* __restrict__ z,
                                                            AdochArgs a) {
    if (*a.all_done) return;
    __shared__ double red[7 * R * NW];
    __shared__ int last_flag;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const double c = a.c;
    double acc[7 * R];
#pragma unroll
    for (int q = 0; q < 7 * R; ++q) acc[q] = 0.0;
    // row i's products for every restart are complete in zr: the row's
    // update of the sums (lane `owner` only)
    auto row_done = [&](int64_t i, const double (&zr)[R]) {
        const double hi = FIELD ? static_cast<double>(h[i]) : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t t = i * R + r;
            const double xi = x[t];
            double zi = zr[r];
            if (FIELD) {
                zi = dadd(zi, dmul(hi, x[n * R + r]));
                acc[7 * r + 6] = dadd(acc[7 * r + 6], dmul(hi, xi));
            }
            z[t] = zi;
            const double yi = dadd(xi, dmul(c, dsub(xi, xp[t])));
            const double jy = dsub(dmul(dadd(1.0, c), zi), dmul(c, zp[t]));
            const double x2 = dmul(xi, xi), y2 = dmul(yi, yi);
            acc[7 * r + 0] = dadd(acc[7 * r + 0], dmul(x2, x2));
            acc[7 * r + 1] = dadd(acc[7 * r + 1], x2);
            acc[7 * r + 2] = dadd(acc[7 * r + 2], dmul(xi, zi));
            acc[7 * r + 3] = dadd(acc[7 * r + 3], dmul(y2, y2));
            acc[7 * r + 4] = dadd(acc[7 * r + 4], y2);
            acc[7 * r + 5] = dadd(acc[7 * r + 5], dmul(yi, jy));
        }
    };
    if constexpr (std::is_same<JS, SinJ>::value) {
        constexpr int RW = kSinRows;
        for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * NW + wave) * RW; i0 < n;
             i0 += static_cast<int64_t>(gridDim.x) * NW * RW) {
            double p[RW][R];
#pragma unroll
            for (int w = 0; w < RW; ++w)
#pragma unroll
                for (int r = 0; r < R; ++r) p[w][r] = 0.0;
            lane_rows_sin_walk<RW>(J, i0, n, lane, [&](int64_t j, const double (&sv)[RW], int dr) {
                double xv[R];
#pragma unroll
                for (int r = 0; r < R; ++r) xv[r] = x[j * R + r];
#pragma unroll
                for (int w = 0; w < RW; ++w)
                    if (w != dr) {
#pragma unroll
                        for (int r = 0; r < R; ++r) p[w][r] = dadd(p[w][r], dmul(sv[w], xv[r]));
                    }
            });
#pragma unroll
            for (int w = 0; w < RW; ++w) {
                double zr[R];
#pragma unroll
                for (int r = 0; r < R; ++r) zr[r] = __shfl(wave_sum(p[w][r]), 0, kWave);
                if (lane == w && i0 + w < n) row_done(i0 + w, zr);
            }
        }
    } else {
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * NW + wave; i < n;
             i += static_cast<int64_t>(gridDim.x) * NW) {
            constexpr int U = 8;
            double p[R];
#pragma unroll
            for (int r = 0; r < R; ++r) p[r] = 0.0;
            int64_t j = lane;
            for (; j + (U - 1) * kWave < n; j += U * kWave) {
                double jv[U], xv[U][R];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    jv[u] = J(i, j + u * kWave);
#pragma unroll
                    for (int r = 0; r < R; ++r) xv[u][r] = x[(j + u * kWave) * R + r];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) p[r] = dadd(p[r], dmul(jv[u], xv[u][r]));
            }
            for (; j < n; j += kWave) {
                const double jv = J(i, j);
#pragma unroll
                for (int r = 0; r < R; ++r) p[r] = dadd(p[r], dmul(jv, x[j * R + r]));
            }
            double zr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) zr[r] = wave_sum(p[r]);
            if (lane == 0) row_done(i, zr);
        }
    }
    block_sum<7 * R, NT>(acc, red);
    adoch_mv_close<R, NT, FIELD>(acc, red, &last_flag, n, x, xp, zp, z, a);
}

int grid_for_rows(int64_t n) {
    int64_t g = (n + NW - 1) / NW;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

int grid_for_elems(int64_t total) {
    int64_t g = (total + NT - 1) / NT;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

int dense_step_grid(int64_t n) { return grid_for_rows(n); }

// Call f with the view's coupling source (stored or procedural).
#define DOCH_WITH_JSRC(A, ...)                                                  \
    do {                                                                        \
        if ((A).proc_kind == 1) {                                               \
            const SinJ js{(A).proc_seed};                                       \
            __VA_ARGS__;                                                        \
        } else {                                                                \
            const StoredJ js{(A).J, (A).ld};                                    \
            __VA_ARGS__;                                                        \
        }                                                                       \
    } while (0)

int adoch_dense_grid(const DenseView& A) {
    const int64_t rows_per_wave = A.proc_kind == 1 ? kSinRows : 1;
    int64_t g = (A.n + NW * rows_per_wave - 1) / (NW * rows_per_wave);
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

hipError_t launch_adoch_dense_mv(const DenseView& A, const double* x, const double* xp, const double* zp,
                                 double* z, const AdochArgs& a, hipStream_t s) {
    const int grid = adoch_dense_grid(A);
    auto go = [&](auto rtag) {
        constexpr int RR = decltype(rtag)::value;
        DOCH_WITH_JSRC(A, {
            using JS = std::decay_t<decltype(js)>;
            if (!A.h)
                hipLaunchKernelGGL((adoch_dense_mv_kernel<double, false, JS, RR>), dim3(grid), dim3(NT), 0, s, A.n,
                                   js, static_cast<const double*>(nullptr), x, xp, zp, z, a);
            else if (A.ht == ISING_F64)
                hipLaunchKernelGGL((adoch_dense_mv_kernel<double, true, JS, RR>), dim3(grid), dim3(NT), 0, s, A.n,
                                   js, static_cast<const double*>(A.h), x, xp, zp, z, a);
            else
                hipLaunchKernelGGL((adoch_dense_mv_kernel<float, true, JS, RR>), dim3(grid), dim3(NT), 0, s, A.n,
                                   js, static_cast<const float*>(A.h), x, xp, zp, z, a);
        });
        return hipGetLastError();
    };
    using std::integral_constant;
    switch (a.R) {
        case 1: return go(integral_constant<int, 1>());
        case 2: return go(integral_constant<int, 2>());
        case 4: return go(integral_constant<int, 4>());
        case 8: return go(integral_constant<int, 8>());
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dense_step(const DenseView& A, const StepArgs& a, int grid, hipStream_t s) {
    const bool field = A.h != nullptr;
    DOCH_WITH_JSRC(A, {
        using JS = std::decay_t<decltype(js)>;
        if (a.x_dtype == ISING_F64) {
            if (!field)
                hipLaunchKernelGGL((dense_step_kernel<double, double, false, JS>), dim3(grid), dim3(NT), 0, s,
                                   A.n, js, static_cast<const double*>(nullptr), a);
            else if (A.ht == ISING_F64)
                hipLaunchKernelGGL((dense_step_kernel<double, double, true, JS>), dim3(grid), dim3(NT), 0, s,
                                   A.n, js, static_cast<const double*>(A.h), a);
            else
                hipLaunchKernelGGL((dense_step_kernel<double, float, true, JS>), dim3(grid), dim3(NT), 0, s,
                                   A.n, js, static_cast<const float*>(A.h), a);
        } else {
            if (!field)
                hipLaunchKernelGGL((dense_step_kernel<float, double, false, JS>), dim3(grid), dim3(NT), 0, s,
                                   A.n, js, static_cast<const double*>(nullptr), a);
            else if (A.ht == ISING_F64)
                hipLaunchKernelGGL((dense_step_kernel<float, double, true, JS>), dim3(grid), dim3(NT), 0, s,
                                   A.n, js, static_cast<const double*>(A.h), a);
            else
                hipLaunchKernelGGL((dense_step_kernel<float, float, true, JS>), dim3(grid), dim3(NT), 0, s,
                                   A.n, js, static_cast<const float*>(A.h), a);
        }
    });
    return hipGetLastError();
}

hipError_t launch_dense_energy(const DenseView& A, const int8_t* s_spins, int R,
                               double* partials, unsigned int* ticket, int grid, double* E,
                               hipStream_t s) {
    if (A.proc_kind == 1 && A.h == nullptr) {
        // procedural couplings: the generator once per block of up to 8
        // restarts (at n = 65536 about 2.5 ms per block of 8, against 26 ms
        // per 64 restarts for the tiled kernel's sine per coupling);
        // partials: R x grid doubles; one ticket per column block
        const SinJ js{A.proc_seed};
        const int RB = R == 1 ? 1 : R == 2 ? 2 : R <= 4 ? 4 : 8;
        const dim3 g(static_cast<unsigned>(grid), static_cast<unsigned>((R + RB - 1) / RB));
        const bool packed = R % 8 == 0 && (reinterpret_cast<uintptr_t>(s_spins) & 7) == 0;
        switch (RB) {
        case 1: hipLaunchKernelGGL((dense_sin_energy_kernel<1, false>), g, dim3(NT), 0, s, A.n, js, s_spins, R, partials, ticket, E); break;
        case 2: hipLaunchKernelGGL((dense_sin_energy_kernel<2, false>), g, dim3(NT), 0, s, A.n, js, s_spins, R, partials, ticket, E); break;
        case 4: hipLaunchKernelGGL((dense_sin_energy_kernel<4, false>), g, dim3(NT), 0, s, A.n, js, s_spins, R, partials, ticket, E); break;
        default:
            if (packed)
                hipLaunchKernelGGL((dense_sin_energy_kernel<8, true>), g, dim3(NT), 0, s, A.n, js, s_spins, R, partials, ticket, E);
            else
                hipLaunchKernelGGL((dense_sin_energy_kernel<8, false>), g, dim3(NT), 0, s, A.n, js, s_spins, R, partials, ticket, E);
            break;
        }
        return hipGetLastError();
    }
    if (R >= kTiledEnergyMinR) {
        // partials: (row tiles) x (R rounded up to 64) x 2 doubles
        const int Rp = (R + 63) / 64 * 64;
        const dim3 tg(static_cast<unsigned>((A.n + 63) / 64), static_cast<unsigned>(Rp / 64));
        DOCH_WITH_JSRC(A, {
            using JS = std::decay_t<decltype(js)>;
            if (A.h == nullptr)
                hipLaunchKernelGGL((dense_energy_tiled_kernel<double, false, JS>), tg, dim3(NT), 0, s, A.n, js,
                                   static_cast<const double*>(nullptr), s_spins, R, Rp, partials, ticket, E);
            else if (A.ht == ISING_F64)
                hipLaunchKernelGGL((dense_energy_tiled_kernel<double, true, JS>), tg, dim3(NT), 0, s, A.n, js,
                                   static_cast<const double*>(A.h), s_spins, R, Rp, partials, ticket, E);
            else
                hipLaunchKernelGGL((dense_energy_tiled_kernel<float, true, JS>), tg, dim3(NT), 0, s, A.n, js,
                                   static_cast<const float*>(A.h), s_spins, R, Rp, partials, ticket, E);
        });
        return hipGetLastError();
    }
    DOCH_WITH_JSRC(A, {
        using JS = std::decay_t<decltype(js)>;
        if (A.h == nullptr)
            hipLaunchKernelGGL((dense_energy_kernel<double, false, JS>), dim3(grid, R), dim3(NT), 0, s,
                               A.n, js, static_cast<const double*>(nullptr), s_spins, R, partials, ticket, E);
        else if (A.ht == ISING_F64)
            hipLaunchKernelGGL((dense_energy_kernel<double, true, JS>), dim3(grid, R), dim3(NT), 0, s,
                               A.n, js, static_cast<const double*>(A.h), s_spins, R, partials, ticket, E);
        else
            hipLaunchKernelGGL((dense_energy_kernel<float, true, JS>), dim3(grid, R), dim3(NT), 0, s,
                               A.n, js, static_cast<const float*>(A.h), s_spins, R, partials, ticket, E);
    });
    return hipGetLastError();
}

hipError_t launch_dense_validate(const DenseView& A, int32_t* flags, hipStream_t s) {
    hipLaunchKernelGGL(dense_validate_kernel, dim3(grid_for_elems(A.n * A.n)), dim3(NT), 0, s,
                       A.n, A.ld, A.J, flags);
    return hipGetLastError();
}

hipError_t launch_dense_symcheck(const DenseView& A, int32_t* bad, hipStream_t s) {
    hipLaunchKernelGGL(dense_symcheck_kernel, dim3(grid_for_elems(A.n * A.n)), dim3(NT), 0, s,
                       A.n, A.ld, A.J, bad);
    return hipGetLastError();
}

hipError_t launch_dense_stats(const DenseView& A, double mean, int pass, double* partials,
                              unsigned int* ticket, int grid, MatrixStats* out, hipStream_t s) {
    DOCH_WITH_JSRC(A, {
        using JS = std::decay_t<decltype(js)>;
        if (A.h == nullptr)
            hipLaunchKernelGGL((dense_stats_kernel<double, false, JS>), dim3(grid), dim3(NT), 0, s, A.n, js,
                               static_cast<const double*>(nullptr), mean, pass, partials, ticket, out);
        else if (A.ht == ISING_F64)
            hipLaunchKernelGGL((dense_stats_kernel<double, true, JS>), dim3(grid), dim3(NT), 0, s, A.n, js,
                               static_cast<const double*>(A.h), mean, pass, partials, ticket, out);
        else
            hipLaunchKernelGGL((dense_stats_kernel<float, true, JS>), dim3(grid), dim3(NT), 0, s, A.n, js,
                               static_cast<const float*>(A.h), mean, pass, partials, ticket, out);
    });
    return hipGetLastError();
}

hipError_t launch_dense_power_step(const DenseView& A, double c, const double* v, double* w,
                                   double* partials, unsigned int* ticket, int grid,
                                   double* mu_log, int64_t k, hipStream_t s) {
    DOCH_WITH_JSRC(A, {
        using JS = std::decay_t<decltype(js)>;
        if (A.h == nullptr)
            hipLaunchKernelGGL((dense_power_kernel<double, false, JS>), dim3(grid), dim3(NT), 0, s, A.n, js,
                               static_cast<const double*>(nullptr), c, v, w, partials, ticket, mu_log, k);
        else if (A.ht == ISING_F64)
            hipLaunchKernelGGL((dense_power_kernel<double, true, JS>), dim3(grid), dim3(NT), 0, s, A.n, js,
                               static_cast<const double*>(A.h), c, v, w, partials, ticket, mu_log, k);
        else
            hipLaunchKernelGGL((dense_power_kernel<float, true, JS>), dim3(grid), dim3(NT), 0, s, A.n, js,
                               static_cast<const float*>(A.h), c, v, w, partials, ticket, mu_log, k);
    });
    return hipGetLastError();
}

}  // namespace doch
