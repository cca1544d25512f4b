// kernels_mfma.hip -- dense J times a block of R restarts on the matrix cores.
//
// With R restarts the DOCH matvec becomes Z = J U, a dense (n x n) by (n x R)
// product with reuse, which belongs on MFMA.  The iteration runs on
// u = sqrt(beta) x, for which eq:FPE reads u <- cbrt(J u + alpha u) (beta
// drops out exactly), so the iterate stays O(sqrt(alpha + lambda)) and is
// representable in BF16 and in FP8 (e4m3, largest finite 448).
//
// One launch per iteration: a workgroup owns a 64 x 64 tile of Z (64 rows,
// 64 restarts), four wavefronts each a 32 x 32 MFMA accumulator.  The
// operands are staged through LDS in 128-byte rows (64 BF16 or 128 FP8 along
// k) padded to 144 bytes so the MFMA fragment reads of 32 rows hit distinct
// banks; the next stage is fetched into registers while the current one is
// multiplied.  J sits in a BF16 copy, or an FP8 copy with one FP32 scale per
// row (J_ij ~ s_i q_ij, s_i = max_j |J_ij| / 448).  The restart block sits as
// an FP32 master (n x R) plus a low-precision transposed copy (R x n) that
// feeds the next product.  In FP8 that copy carries one FP32 scale per
// restart, c_j, with |u_ij| <= 448 c_j: exact at the start (column maximum)
// and carried forward by the bound |u'| = |cbrt(z + alpha u)| <=
// cbrt((rho_q + alpha) M) for |u| <= M, where rho_q is the largest absolute
// row sum of the quantised J.  The bound tends to sqrt(rho_q + alpha), so
// large starting points (u = sqrt(beta) x is large when beta is) never reach
// the format's overflow, and later steps keep its full relative precision.  The epilogue applies the update in FP64, stores
// both copies and adds the restart's FP64 partial sums; the last workgroup
// closes the iteration for every restart (H, r, freezing at r < eps).
#include "device_common.h"
#include "ising_internal.h"

namespace doch {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MT = 256;        // threads per workgroup
constexpr int ROWB = 144;      // staged row: 128 bytes of k plus 16 bytes of pad

template <int PREC> struct Prec;
template <> struct Prec<0> {   // BF16
    using T = __bf16;
    static constexpr int KT = 64;
};
template <> struct Prec<1> {   // FP8 e4m3 (OCP)
    using T = uint8_t;
    static constexpr int KT = 128;
};

constexpr float kFp8Max = 448.0f;
// margin on the carried bound: FP32 accumulation of the product (relative
// error below n 2^-24 <= 2^-8 for n <= 65536) and rounding of the update
constexpr double kBoundSlack = 1.01;

__device__ __forceinline__ uint8_t to_fp8(float f) {
    // v_cvt_pk_fp8_f32 rounds to nearest even; the operands are scaled into
    // range, the clamp only guards the boundary
    f = fminf(fmaxf(f, -kFp8Max), kFp8Max);
    return static_cast<uint8_t>(__builtin_amdgcn_cvt_pk_fp8_f32(f, 0.0f, 0, false) & 0xff);
}

// OCP e4m3 code -> value: bias 7, 3 mantissa bits, subnormals at exponent 0
__device__ __forceinline__ double fp8_value(uint8_t q) {
    const int e = (q >> 3) & 15, m = q & 7;
    const double mag = e == 0 ? ldexp(static_cast<double>(m), -9) : ldexp(1.0 + m / 8.0, e - 7);
    return (q & 0x80) ? -mag : mag;
}

// carried bound of the next iterate's magnitude, as a restart scale
__device__ __forceinline__ float next_colscale(float c_old, double rho_q, double alpha) {
    const double m_old = dmul(static_cast<double>(kFp8Max), static_cast<double>(c_old));
    const double m_new = dmul(kBoundSlack, cbrt(dmul(dadd(dmul(kBoundSlack, rho_q), alpha), m_old)));
    return static_cast<float>(dmul(ddiv(m_new, static_cast<double>(kFp8Max)), kBoundSlack));
}

template <int PREC>
__device__ __forceinline__ typename Prec<PREC>::T to_lowp(float f) {
    if constexpr (PREC == 0) return static_cast<__bf16>(f);
    else return to_fp8(f);
}

// One MFMA step on fragments read from the staged tiles.  a_row / b_row
// point at this lane's staged row; koff is the element offset along k.
template <int PREC>
__device__ __forceinline__ f32x16 mfma_step(const char* a_row, const char* b_row, int koff, f32x16 c) {
    if constexpr (PREC == 0) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(a_row + 2 * koff);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(b_row + 2 * koff);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    } else {
        const long a = *reinterpret_cast<const long*>(a_row + koff);
        const long b = *reinterpret_cast<const long*>(b_row + koff);
        return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, c, 0, 0, 0);
    }
}

template <int PREC>
__global__ __launch_bounds__(MT) void lowp_step_kernel(
    int np, int Rp, const typename Prec<PREC>::T* __restrict__ Jq, const float* __restrict__ rscale,
    const float* __restrict__ U_old, float* __restrict__ U_new,
    const typename Prec<PREC>::T* __restrict__ Ub_old, typename Prec<PREC>::T* __restrict__ Ub_new,
    const float* __restrict__ cs_old, float* __restrict__ cs_new, double rho_q,
    double alpha, double beta, double eps, int R, int64_t k, double* __restrict__ partials,
    unsigned int* ticket, double* __restrict__ log, RestartState* __restrict__ state) {
    using T = typename Prec<PREC>::T;
    constexpr int KT = Prec<PREC>::KT;
    __shared__ __attribute__((aligned(16))) char sA[64 * ROWB];
    __shared__ __attribute__((aligned(16))) char sB[64 * ROWB];
    __shared__ double red[2][64][4];
    __shared__ int last_flag;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int row0 = blockIdx.x * 64;
    const int col0 = blockIdx.y * 64;
    // global -> register staging: thread loads 16-byte chunks c = tid, tid+256
    // of the 64 x 128-byte tile (row = c / 8, chunk = c % 8)
    const char* gA = reinterpret_cast<const char*>(Jq) + static_cast<size_t>(row0) * np * sizeof(T);
    const char* gB = reinterpret_cast<const char*>(Ub_old) + static_cast<size_t>(col0) * np * sizeof(T);
    const size_t gstride = static_cast<size_t>(np) * sizeof(T);
    i32x4 ra[2], rb[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = tid + MT * u;
            const int r = c >> 3, ch = c & 7;
            const size_t off = r * gstride + static_cast<size_t>(k0) * sizeof(T) + ch * 16;
            ra[u] = *reinterpret_cast<const i32x4*>(gA + off);
            rb[u] = *reinterpret_cast<const i32x4*>(gB + off);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = tid + MT * u;
            const int r = c >> 3, ch = c & 7;
            *reinterpret_cast<i32x4*>(sA + r * ROWB + ch * 16) = ra[u];
            *reinterpret_cast<i32x4*>(sB + r * ROWB + ch * 16) = rb[u];
        }
    };
    f32x16 acc = {};
    const char* a_row = sA + (wr * 32 + (lane & 31)) * ROWB;
    const char* b_row = sB + (wc * 32 + (lane & 31)) * ROWB;
    const int khalf = (lane >> 5) * 8;          // this lane's 8 consecutive k of a 16-deep step
    fetch(0);
    for (int k0 = 0; k0 < np; k0 += KT) {
        stash();
        __syncthreads();
        if (k0 + KT < np) fetch(k0 + KT);
#pragma unroll
        for (int kk = 0; kk < KT; kk += 16) acc = mfma_step<PREC>(a_row, b_row, kk + khalf, acc);
        __syncthreads();
    }
    // ---- epilogue: lane holds column j, rows 8*(v/4) + 4*(lane/32) + v%4
    const int j = col0 + wc * 32 + (lane & 31);
    const bool live = j < R && !state[j < R ? j : 0].done;
    double part[4] = {0.0, 0.0, 0.0, 0.0};      // u^4, u^2, u z, (du)^2
    // FP8: scale of the copy read by this product and of the one written now
    float c_in = 1.0f, c_out = 1.0f;
    if constexpr (PREC == 1) {
        c_in = cs_old[j];
        c_out = live ? next_colscale(c_in, rho_q, alpha) : c_in;
        if (blockIdx.x == 0 && wr == 0 && lane < 32) cs_new[j] = c_out;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = row0 + wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const size_t ij = static_cast<size_t>(i) * Rp + j;
        const double uo = static_cast<double>(U_old[ij]);
        double z = static_cast<double>(acc[v]);
        if (PREC == 1) z = dmul(dmul(z, static_cast<double>(rscale[i])), static_cast<double>(c_in));
        float un = static_cast<float>(uo);
        if (live) {
            un = static_cast<float>(cbrt(dadd(z, dmul(alpha, uo))));
            const double d = dsub(static_cast<double>(un), uo);
            const double u2 = dmul(uo, uo);
            part[0] = dadd(part[0], dmul(u2, u2));
            part[1] = dadd(part[1], u2);
            part[2] = dadd(part[2], dmul(uo, z));
            part[3] = dadd(part[3], dmul(d, d));
        }
        U_new[ij] = un;
        Ub_new[static_cast<size_t>(j) * np + i] = to_lowp<PREC>(PREC == 1 ? un / c_out : un);
    }
    // rows of a column: lanes l and l + 32, then the two row halves of the tile
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q] = dadd(part[q], __shfl_xor(part[q], 32, 64));
    if (lane < 32) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wr][wc * 32 + lane][q] = part[q];
    }
    __syncthreads();
    if (tid < 64) {
        double* p = partials + (static_cast<size_t>(blockIdx.x) * Rp + col0 + tid) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) store_agent(p + q, dadd(red[0][tid][q], red[1][tid][q]));
    }
    __syncthreads();
    if (tid == 0) last_flag = arrive_last(ticket, gridDim.x * gridDim.y) ? 1 : 0;
    __syncthreads();
    if (!last_flag) return;
    // ---- last workgroup: close the iteration of every live restart
    for (int c = tid; c < R; c += MT) {
        if (state[c].done) continue;
        double S[4] = {0.0, 0.0, 0.0, 0.0};
        for (unsigned t = 0; t < gridDim.x; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                S[q] = dadd(S[q], load_agent(partials + (static_cast<size_t>(t) * Rp + c) * 4 + q));
        // H(x) = H_u / beta with x = u / sqrt(beta); r is scale free
        const double Hu = dsub(dsub(dmul(0.25, S[0]), dmul(ddiv(alpha, 2.0), S[1])), dmul(0.5, S[2]));
        const double H = ddiv(Hu, beta);
        const double r = S[1] == 0.0 ? 0.0 : ddiv(sqrt(S[3]), sqrt(S[1]));
        log[(static_cast<size_t>(k) * R + c) * 2] = H;
        log[(static_cast<size_t>(k) * R + c) * 2 + 1] = r;
        RestartState& st = state[c];
        st.iters_done = k + 1;
        st.H_last = H;
        st.r_last = r;
        if (!isfinite(H) || !isfinite(r)) {
            st.nonfinite = 1;
            st.done = 1;
        } else if (eps > 0.0 && r < eps) {
            st.converged = 1;
            st.done = 1;
        }
    }
    if (tid == 0) reset_ticket(ticket);
}

__device__ __forceinline__ float start_u(const double* x0, int64_t i, int R, int j, double sqrt_beta) {
    return static_cast<float>(dmul(x0[i * R + j], sqrt_beta));
}

// FP8: max_i |u_ij| of the starting block, as float bits (order-preserving
// for non-negative values), combined over row chunks of 64 with atomicMax
// into colmax_bits (zeroed by the caller).
__global__ __launch_bounds__(256) void lowp_colmax_kernel(const double* __restrict__ x0, int n, int R,
                                                          double sqrt_beta,
                                                          unsigned int* __restrict__ colmax_bits) {
    const int j = blockIdx.y * 256 + threadIdx.x;
    if (j >= R) return;
    const int i0 = blockIdx.x * 64;
    const int i1 = i0 + 64 < n ? i0 + 64 : n;
    float m = 0.0f;
    for (int i = i0; i < i1; ++i) m = fmaxf(m, fabsf(start_u(x0, i, R, j, sqrt_beta)));
    atomicMax(colmax_bits + j, __float_as_uint(m));
}

// x0 (n x R, double) -> u = sqrt(beta) x in the padded FP32 master and the
// transposed low-precision copy; padding rows and restarts are zero.  FP8
// divides by the restart scale c_j = max_i |u_ij| / 448 (1 for a zero
// column) and records it.
template <int PREC>
__global__ __launch_bounds__(256) void lowp_load_kernel(const double* __restrict__ x0, int n, int R,
                                                       int np, int Rp, double sqrt_beta,
                                                       const unsigned int* __restrict__ colmax_bits,
                                                       float* __restrict__ cs, float* __restrict__ U,
                                                       typename Prec<PREC>::T* __restrict__ Ub) {
    const int64_t total = static_cast<int64_t>(np) * Rp;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * 256) {
        const int i = static_cast<int>(t / Rp), j = static_cast<int>(t % Rp);
        const float u = (i < n && j < R) ? start_u(x0, i, R, j, sqrt_beta) : 0.0f;
        U[t] = u;
        if constexpr (PREC == 1) {
            const float m = j < R ? __uint_as_float(colmax_bits[j]) : 0.0f;
            const float c = m > 0.0f ? m / kFp8Max : 1.0f;
            if (i == 0) cs[j] = c;
            Ub[static_cast<int64_t>(j) * np + i] = to_fp8(u / c);
        } else {
            Ub[static_cast<int64_t>(j) * np + i] = to_lowp<PREC>(u);
        }
    }
}

// u -> x = u / sqrt(beta) (double) and sign(x).
__global__ __launch_bounds__(256) void lowp_finish_kernel(const float* __restrict__ U, int n, int R,
                                                          int Rp, double sqrt_beta,
                                                          double* __restrict__ x_out,
                                                          int8_t* __restrict__ s_out) {
    const int64_t total = static_cast<int64_t>(n) * R;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * 256) {
        const int i = static_cast<int>(t / R), j = static_cast<int>(t % R);
        const double x = ddiv(static_cast<double>(U[static_cast<int64_t>(i) * Rp + j]), sqrt_beta);
        if (x_out) x_out[t] = x;
        if (s_out) s_out[t] = x >= 0.0 ? 1 : -1;
    }
}

// FP64 J -> padded BF16 copy, or FP8 copy with per-row scales and the
// absolute row sums s_i sum_j |q_ij| of the quantised rows (rowabs).
template <int PREC>
__global__ __launch_bounds__(256) void lowp_convert_kernel(const double* __restrict__ J, int n, int np,
                                                           typename Prec<PREC>::T* __restrict__ Jq,
                                                           float* __restrict__ rscale,
                                                           double* __restrict__ rowabs) {
    __shared__ double red[4];
    for (int i = blockIdx.x; i < np; i += gridDim.x) {
        float s = 1.0f;
        if (PREC == 1) {
            double m = 0.0;
            if (i < n)
                for (int c = threadIdx.x; c < n; c += 256) m = fmax(m, fabs(J[static_cast<int64_t>(i) * n + c]));
            m = wave_max(m);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
            __syncthreads();
            m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            __syncthreads();
            s = m > 0.0 ? static_cast<float>(m / 448.0) : 1.0f;
            if (threadIdx.x == 0) rscale[i] = s;
        }
        double ra = 0.0;
        for (int c = threadIdx.x; c < np; c += 256) {
            const double v = (i < n && c < n) ? J[static_cast<int64_t>(i) * n + c] : 0.0;
            if constexpr (PREC == 1) {
                const uint8_t q = to_fp8(static_cast<float>(v / static_cast<double>(s)));
                Jq[static_cast<int64_t>(i) * np + c] = q;
                ra = dadd(ra, fabs(fp8_value(q)));
            } else {
                Jq[static_cast<int64_t>(i) * np + c] = to_lowp<PREC>(static_cast<float>(v));
            }
        }
        if constexpr (PREC == 1) {
            ra = wave_sum(ra);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ra;
            __syncthreads();
            if (threadIdx.x == 0)
                rowabs[i] = dmul(dadd(dadd(red[0], red[1]), dadd(red[2], red[3])), static_cast<double>(s));
            __syncthreads();
        }
    }
}

// FP64 objective of R final iterates with the FP64 J (eq:Hamilton):
// workgroup per (row block, restart); one wavefront per row.
__global__ __launch_bounds__(256) void dense_objective_kernel(const double* __restrict__ J, int n,
                                                              int R, const double* __restrict__ X,
                                                              double alpha, double beta,
                                                              double* __restrict__ partials,
                                                              unsigned int* tickets,
                                                              double* __restrict__ H) {
    __shared__ double red[3 * 4];
    __shared__ int last_flag;
    const int r = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[3] = {0.0, 0.0, 0.0};                 // x^4, x^2, x (J x)
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + wave; i < n;
         i += static_cast<int64_t>(gridDim.x) * 4) {
        double p = 0.0;
        for (int c = lane; c < n; c += 64) p = dadd(p, dmul(J[i * n + c], X[static_cast<int64_t>(c) * R + r]));
        const double z = wave_sum(p);
        if (lane == 0) {
            const double xi = X[i * R + r];
            const double x2 = dmul(xi, xi);
            v[0] = dadd(v[0], dmul(x2, x2));
            v[1] = dadd(v[1], x2);
            v[2] = dadd(v[2], dmul(xi, z));
        }
    }
    block_sum<3, 256>(v, red);
    double* p = partials + (static_cast<size_t>(r) * gridDim.x + blockIdx.x) * 3;
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q) store_agent(p + q, v[q]);
        last_flag = arrive_last(tickets + r, gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!last_flag) return;
    double u[3] = {0.0, 0.0, 0.0};
    const double* pr = partials + static_cast<size_t>(r) * gridDim.x * 3;
    for (unsigned g = threadIdx.x; g < gridDim.x; g += 256)
        for (int q = 0; q < 3; ++q) u[q] = dadd(u[q], load_agent(pr + g * 3 + q));
    block_sum<3, 256>(u, red);
    if (threadIdx.x == 0) {
        H[r] = dsub(dsub(dmul(ddiv(beta, 4.0), u[0]), dmul(ddiv(alpha, 2.0), u[1])), dmul(0.5, u[2]));
        reset_ticket(tickets + r);
    }
}

}  // namespace

hipError_t launch_lowp_convert(int prec, const double* J, int n, int np, void* Jq, float* rscale,
                               double* rowabs, hipStream_t s) {
    const int grid = np < 4096 ? np : 4096;
    if (prec == 0)
        hipLaunchKernelGGL(lowp_convert_kernel<0>, dim3(grid), dim3(256), 0, s, J, n, np,
                           static_cast<__bf16*>(Jq), rscale, rowabs);
    else
        hipLaunchKernelGGL(lowp_convert_kernel<1>, dim3(grid), dim3(256), 0, s, J, n, np,
                           static_cast<uint8_t*>(Jq), rscale, rowabs);
    return hipGetLastError();
}

hipError_t launch_lowp_load(int prec, const double* x0, int n, int R, int np, int Rp, double sqrt_beta,
                            unsigned int* colmax_bits, float* cs, float* U, void* Ub, hipStream_t s) {
    int64_t g = (static_cast<int64_t>(np) * Rp + 255) / 256;
    if (g > 8192) g = 8192;
    if (prec == 0) {
        hipLaunchKernelGGL(lowp_load_kernel<0>, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, x0, n, R,
                           np, Rp, sqrt_beta, nullptr, nullptr, U, static_cast<__bf16*>(Ub));
    } else {
        hipError_t e = hipMemsetAsync(colmax_bits, 0, static_cast<size_t>(R) * sizeof(unsigned int), s);
        if (e != hipSuccess) return e;
        const dim3 cg((n + 63) / 64, (R + 255) / 256);
        hipLaunchKernelGGL(lowp_colmax_kernel, cg, dim3(256), 0, s, x0, n, R, sqrt_beta, colmax_bits);
        hipLaunchKernelGGL(lowp_load_kernel<1>, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, x0, n, R,
                           np, Rp, sqrt_beta, colmax_bits, cs, U, static_cast<uint8_t*>(Ub));
    }
    return hipGetLastError();
}

hipError_t launch_lowp_step(int prec, int np, int Rp, const void* Jq, const float* rscale,
                            const float* U_old, float* U_new, const void* Ub_old, void* Ub_new,
                            const float* cs_old, float* cs_new, double rho_q,
                            double alpha, double beta, double eps, int R, int64_t k,
                            double* partials, unsigned int* ticket, double* log, RestartState* state,
                            hipStream_t s) {
    const dim3 grid(np / 64, Rp / 64);
    if (prec == 0)
        hipLaunchKernelGGL(lowp_step_kernel<0>, grid, dim3(MT), 0, s, np, Rp,
                           static_cast<const __bf16*>(Jq), rscale, U_old, U_new,
                           static_cast<const __bf16*>(Ub_old), static_cast<__bf16*>(Ub_new), cs_old,
                           cs_new, rho_q, alpha, beta, eps, R, k, partials, ticket, log, state);
    else
        hipLaunchKernelGGL(lowp_step_kernel<1>, grid, dim3(MT), 0, s, np, Rp,
                           static_cast<const uint8_t*>(Jq), rscale, U_old, U_new,
                           static_cast<const uint8_t*>(Ub_old), static_cast<uint8_t*>(Ub_new), cs_old,
                           cs_new, rho_q, alpha, beta, eps, R, k, partials, ticket, log, state);
    return hipGetLastError();
}

hipError_t launch_lowp_finish(const float* U, int n, int R, int Rp, double sqrt_beta, double* x_out,
                              int8_t* s_out, hipStream_t s) {
    int64_t g = (static_cast<int64_t>(n) * R + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(lowp_finish_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, U, n, R, Rp,
                       sqrt_beta, x_out, s_out);
    return hipGetLastError();
}

hipError_t launch_dense_objective(const double* J, int n, int R, const double* X, double alpha,
                                  double beta, double* partials, unsigned int* tickets, int grid,
                                  double* H, hipStream_t s) {
    hipLaunchKernelGGL(dense_objective_kernel, dim3(grid, R), dim3(256), 0, s, J, n, R, X, alpha, beta,
                       partials, tickets, H);
    return hipGetLastError();
}

}  // namespace doch
